"""Host-side checks of the butterfly precompute (Sec. 3.1-3.2): the
interpolative decomposition and the compressed operator, evaluated on the
host from the plan's records, against the oracle's Legendre values.

These run without a GPU (host-only plans).  Pins:
* the ID satisfies the bound of Sec. 3.1 (Eq. 20) with the singular values
  numpy's SVD gives, reproduces an exactly low-rank matrix, and keeps the
  rank scipy's ID library finds at the same tolerance (within one);
* the compressed Lambda^T x equals the dense one (long-double oracle
  Legendre values) within a few eps at every level count.
"""
import numpy as np
import pytest

import oracle
from paper_1110_4874_amd import sht


@pytest.fixture(scope="module")
def lib():
    return sht.load()


def _legendre_block(L, N, m, t, rows, cols):
    return np.array([oracle.plm_ring(L, m, N, k + 1, ld=True)[t::2][rows] for k in cols]).T


@pytest.mark.parametrize("tol", [1e-6, 1e-10, 1e-13])
@pytest.mark.parametrize("m,t,r0,c0", [(10, 0, 100, 64), (200, 1, 40, 300), (0, 0, 0, 0)])
def test_interp_decomp_bound(lib, tol, m, t, r0, c0):
    L, N = 511, 256
    A = _legendre_block(L, N, m, t, slice(r0, r0 + 96), range(c0, c0 + 64))
    k, piv, T = sht.interp_decomp(A, tol)
    c = A.shape[1]
    assert sorted(piv.tolist()) == list(range(c))
    R = A[:, piv[k:]] - A[:, piv[:k]] @ T
    s = np.linalg.svd(A, compute_uv=False)
    sk = s[k] if k < len(s) else 0.0
    err = np.linalg.norm(R, 2) if k < c else 0.0
    assert err <= np.sqrt(4 * k * (c - k) + 1) * sk + 1e-15 * s[0]
    assert err <= 4 * tol * np.sqrt(c) * s[0]
    assert np.abs(T).max(initial=0.0) <= 4.0


def test_interp_decomp_exact_low_rank(lib):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((80, 5)) @ rng.standard_normal((5, 40))
    k, piv, T = sht.interp_decomp(A, 1e-12)
    assert k == 5
    R = A[:, piv[k:]] - A[:, piv[:k]] @ T
    assert np.abs(R).max() <= 1e-12 * np.abs(A).max()


def test_interp_decomp_rank_matches_scipy(lib):
    sli = pytest.importorskip("scipy.linalg.interpolative")
    L, N = 511, 256
    for (m, t, r0, c0) in [(10, 0, 100, 64), (60, 1, 0, 128)]:
        A = _legendre_block(L, N, m, t, slice(r0, r0 + 128), range(c0, c0 + 64))
        for tol in (1e-8, 1e-12):
            k, _, _ = sht.interp_decomp(A, tol)
            ks, _, _ = sli.interp_decomp(A.copy(), tol)
            assert abs(k - ks) <= 1, (m, t, tol, k, ks)


def _dense_apply(L, N, m, t, x):
    n = len(x)
    return np.array([np.dot(oracle.plm_ring(L, m, N, k + 1, ld=True)[t::2][:n], x) for k in range(2 * N)])


@pytest.mark.parametrize("L,N,eps,levels,batch", [(255, 128, 1e-12, 3, 0), (255, 128, 1e-8, 2, 1),
                                                  (127, 64, 1e-12, -1, 0), (200, 64, 1e-10, 2, 1),
                                                  (511, 256, 1e-12, 4, 0), (511, 256, 1e-12, 4, 2)])
def test_compressed_operator_matches_dense(lib, L, N, eps, levels, batch):
    p = sht.Plan(L, N, eps, host_only=True, max_levels=levels, batch_mib=batch)
    info = p.info()
    assert info["bf_built"] == 1
    if batch:
        assert info["bf_nbatch"] > 1
    if levels > 0:
        assert p.butterfly_depth(0, 0) == levels
    rng = np.random.default_rng(L)
    worst = 0.0
    for m in [0, 1, 7, L // 4, L // 2, L - 5]:
        for t in (0, 1):
            n = (L - m - t) // 2 + 1
            x = rng.standard_normal(n)
            y = p.butterfly_apply_host(m, t, x)
            ref = _dense_apply(L, N, m, t, x)
            worst = max(worst, float(np.max(np.abs(y - ref)) / np.max(np.abs(ref))))
    print(f"L={L} eps={eps} levels={levels} worst rel err {worst:.2e}")
    assert worst <= 8 * eps + 2e-12


def test_depth_zero_and_histogram(lib):
    L, N = 127, 64
    p0 = sht.Plan(L, N, 1e-12, host_only=True, max_levels=0)
    inf = p0.info()
    assert inf["bf_T_entries"] == 0
    assert inf["bf_depth_hist"][0] == 2 * (L + 1)
    assert inf["bf_res_elems"] == inf["n_step_exec"]
    p2 = sht.Plan(L, N, 1e-12, host_only=True, max_levels=2)
    hist = p2.info()["bf_depth_hist"]
    assert sum(hist) == 2 * (L + 1)
    assert p2.butterfly_depth(0, 0) == 2


def test_plan_is_deterministic(lib):
    a = sht.Plan(200, 64, 1e-10, host_only=True, max_levels=2).info()
    b = sht.Plan(200, 64, 1e-10, host_only=True, max_levels=2, nthreads=3).info()
    for key in ("bf_T_entries", "bf_res_elems", "bf_nodes", "bf_units", "bf_res_lanes"):
        assert a[key] == b[key]


def test_plan_rejects_column_sets_beyond_the_level_lds():
    # one 512-ring column block at level 1 would need 256 KiB of LDS in the
    # fused level-1 kernel at 8 maps in FP64: refused when the plan is built
    with pytest.raises(sht.ShtError, match="too wide"):
        sht.Plan(511, 256, 1e-10, host_only=True, max_levels=1, chunk=512)
    p = sht.Plan(511, 256, 1e-10, host_only=True, max_levels=1, chunk=128)
    assert p.info()["bf_built"] == 1
