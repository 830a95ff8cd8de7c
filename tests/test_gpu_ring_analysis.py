"""Ring stage of the adjoint on random maps against the transposed ring sum
by its definition (tests/ring_defs.py), both adjoint conventions."""
import numpy as np
import pytest
import torch

import oracle
from ring_defs import ring_direct_adjoint

pytestmark = pytest.mark.gpu

RINGS_2100 = [1, 2, 3, 50, 127, 128, 300, 511, 512, 518, 525, 526, 527, 599, 600, 601, 1200, 1799, 1800,
              1801, 1873, 1874, 1875, 1888, 2398, 2399]


@pytest.mark.parametrize("B,conv", [(1, 0), (2, 0), (3, 1), (4, 0)])
def test_ring_analysis_direct_l2100(gpu, B, conv):
    L, N = 2100, 600
    rng = np.random.default_rng(950 + B)
    maps = rng.standard_normal((B, 12 * N * N))
    p = gpu.Plan(L, N)
    yb = p.ring_analysis(torch.from_numpy(maps).cuda(), convention=conv).cpu().numpy()  # (nrings, L+1, B)
    wpos = 2.0 if conv == gpu.ADJ_TRANSPOSE else 1.0
    worst = 0.0
    for ring in RINGS_2100:
        z, st, J, s, off = oracle.ring_info(N, ring)
        ref = ring_direct_adjoint(maps[:, off:off + J], L, J, s, wpos)
        worst = max(worst, float(np.max(np.abs(yb[ring - 1] - ref)) / np.max(np.abs(ref))))
    print(f"L=2100 N=600 B={B} conv={conv} ring-analysis maxrel={worst:.3e}")
    assert worst <= 1e-12
