"""Pins of the ring-sum definitions the ring-kernel tests compare with
(tests/ring_defs.py): the synthesis sum against the oracle's synthesis on
every ring, and the adjoint sum as its exact transpose."""
import numpy as np

import oracle
from paper_1110_4874_amd.synthetic import alm_gaussian
from ring_defs import ring_direct, ring_direct_adjoint


def test_ring_sum_matches_oracle_synthesis():
    L, N = 40, 16  # rings with J < L, J > L and the belt
    alm = alm_gaussian(L, [7, 8])
    rings = np.arange(1, 4 * N)
    q = oracle.legendre_phase_rings(L, N, alm, rings)
    ref = oracle.synthesis(L, N, alm)
    scale = np.max(np.abs(ref))
    for r in rings:
        z, st, J, s, off = oracle.ring_info(N, int(r))
        assert np.max(np.abs(ring_direct(q[r - 1], J, s) - ref[:, off:off + J])) / scale < 1e-14


def test_ring_adjoint_is_the_transpose():
    rng = np.random.default_rng(5)
    for L, J, s in ((40, 8, 1), (40, 64, 0), (17, 100, 1), (63, 4, 1), (10, 12, 0)):
        q = rng.standard_normal((L + 1, 2)) + 1j * rng.standard_normal((L + 1, 2))
        y = rng.standard_normal((2, J))
        lhs = np.sum(y * ring_direct(q, J, s))
        g = ring_direct_adjoint(y, L, J, s, 2.0)
        rhs = np.sum(q.real * g.real + q.imag * g.imag)
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
        assert np.all(g[0].imag == 0.0)
