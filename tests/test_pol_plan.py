"""Host side of the polarized synthesis: the polar-cap tables and the
host form of the polar spin-2 recurrence, against the oracle's spin-weighted
functions at the exact ring positions (long double)."""
import math

import numpy as np
import pytest

import oracle
from paper_1110_4874_amd import sht


@pytest.fixture(scope="module")
def lib():
    sht.load()
    return sht


def test_polar_ring_count(lib):
    for L, N in ((512, 256), (1024, 512), (96, 48)):
        p = lib.Plan(L, N, host_only=True)
        thr = 0.1 * math.sqrt((L + 1) / 4096.0)
        want = 0
        while want < 2 * N and oracle.ring_info(N, want + 1)[1] < thr:
            want += 1
        assert p.info()["pol_rings"] == want


@pytest.mark.parametrize("L,N", [(512, 256), (1024, 512)])
def test_polar_recurrence_matches_oracle(lib, L, N):
    p = lib.Plan(L, N, host_only=True)
    npol = p.info()["pol_rings"]
    assert npol > 0
    worst = 0.0
    for k in sorted(set([0, 1, npol // 2, npol - 1])):
        for m in (0, 1, 2, 3, 7, 40, 150):
            for s in (2, -2):
                col = p.pol_column_host(m, s, k)
                ref = oracle.spin_ring(L - 1, m, s, N, k + 1)
                sc = np.max(np.abs(ref))
                if sc == 0:
                    assert np.max(np.abs(col)) == 0
                    continue
                worst = max(worst, np.max(np.abs(col - ref)) / sc)
    assert worst < 1e-13


def test_polar_tables_round_trip(lib, tmp_path):
    p = lib.Plan(256, 128, host_only=True)
    path = str(tmp_path / "pol.plan")
    p.save(path)
    q = lib.Plan.load(path, host_only=True)
    assert q.info()["pol_rings"] == p.info()["pol_rings"]
    for m, s, k in ((0, 2, 0), (5, -2, 1), (30, 2, 2)):
        assert np.array_equal(p.pol_column_host(m, s, k), q.pol_column_host(m, s, k))
