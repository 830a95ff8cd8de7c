"""GPU parity of the transposed butterfly (the adjoint through the Sec. 3.2
factorization applied backwards) against the CPU oracle's plain transpose.

FP64 bar: max |g - g_ref| / max |g_ref| per map <= eps + 1e-12, the same bar
as the compressed synthesis.  The transposed butterfly is the exact transpose
of the plan's compressed synthesis, so the dot-product identity
<Y~ a, y> = <a, Y~^T y> holds to rounding (1e-13 of |Y~ a| |y|), which pins
the level and residual transposes independently of the oracle.  FP32 level
products: parity unpinned (no bound from the paper); the measured error is
printed and must stay below 2e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1110_4874_amd import sht
from paper_1110_4874_amd.synthetic import alm_gaussian, gaussian_map

pytestmark = pytest.mark.gpu


def maxrel_cols(g, ref):
    return max(float(np.max(np.abs(g[:, b] - ref[:, b])) / np.max(np.abs(ref[:, b])))
               for b in range(ref.shape[1]))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _maps(N, B, seed0):
    return gaussian_map(12 * N * N, [seed0 + b for b in range(B)])


@pytest.mark.parametrize("L,N,eps,levels,B,batch", [(127, 64, 1e-12, -1, 1, 0), (127, 64, 1e-12, 2, 3, 0),
                                                    (255, 128, 1e-12, 3, 4, 0), (200, 64, 1e-8, 2, 2, 0),
                                                    (511, 256, 1e-12, 4, 1, 0), (300, 128, 1e-10, 3, 9, 0),
                                                    (0, 1, 1e-12, -1, 1, 0), (9, 2, 1e-12, 1, 2, 0),
                                                    (255, 128, 1e-12, 3, 4, 1), (511, 256, 1e-12, 4, 2, 2),
                                                    # passes of several 8-map groups: 16, 16 + 4 + 1, 64,
                                                    # 64 + 8 (two passes), and order batches
                                                    (255, 128, 1e-12, 3, 16, 0), (200, 64, 1e-10, 3, 21, 0),
                                                    (127, 64, 1e-12, 2, 64, 0), (63, 32, 1e-12, 2, 72, 0),
                                                    (255, 128, 1e-12, 3, 24, 1)])
@pytest.mark.parametrize("tr", [False, True])
def test_butterfly_adjoint_parity(gpu, L, N, eps, levels, B, batch, tr):
    maps = _maps(N, B, 700)
    p = gpu.Plan(L, N, eps, max_levels=levels, batch_mib=batch, store_transpose=tr)
    if batch:
        assert p.info()["bf_nbatch"] > 1
    g = p.adjoint(_dev(maps), path=sht.PATH_BUTTERFLY).cpu().numpy()
    ref = oracle.adjoint(L, N, maps)
    err = maxrel_cols(g, ref)
    print(f"L={L} N={N} eps={eps} levels={levels} B={B} transposed copy={tr} "
          f"hist={p.info()['bf_depth_hist'][:6]} adjoint maxrel={err:.3e}")
    assert err <= eps + 1e-12


@pytest.mark.parametrize("prec,tol", [(sht.PREC_FP64, 1e-13), (sht.PREC_FP32, 1e-5)])
@pytest.mark.parametrize("tr", [False, True])
def test_butterfly_adjoint_is_transpose_of_butterfly_synthesis(gpu, prec, tol, tr):
    L, N, B = 255, 128, 3
    alm = alm_gaussian(L, [41, 42, 43])
    maps = _maps(N, B, 720)
    p = gpu.Plan(L, N, 1e-8, max_levels=3, store_fp32=True, store_transpose=tr)
    f = p.synthesis(_dev(alm), path=sht.PATH_BUTTERFLY, precision=prec).cpu().numpy()
    g = p.adjoint(_dev(maps), path=sht.PATH_BUTTERFLY, precision=prec).cpu().numpy()
    for b in range(B):
        lhs = float(np.dot(f[b], maps[b]))
        rhs = float(np.sum(alm[:, b].real * g[:, b].real + alm[:, b].imag * g[:, b].imag))
        scale = float(np.linalg.norm(f[b]) * np.linalg.norm(maps[b]))
        print(f"prec={prec} map {b}: |lhs - rhs| / scale = {abs(lhs - rhs) / scale:.3e}")
        assert abs(lhs - rhs) <= tol * scale, (lhs, rhs)


@pytest.mark.parametrize("tr", [False, True])
def test_butterfly_adjoint_fp32(gpu, tr):
    L, N, B = 255, 128, 4
    maps = _maps(N, B, 740)
    p = gpu.Plan(L, N, 1e-7, max_levels=3, store_fp32=True, store_transpose=tr)
    g32 = p.adjoint(_dev(maps), path=sht.PATH_BUTTERFLY, precision=sht.PREC_FP32).cpu().numpy()
    g64 = p.adjoint(_dev(maps), path=sht.PATH_BUTTERFLY, precision=sht.PREC_FP64).cpu().numpy()
    ref = oracle.adjoint(L, N, maps)
    e32, e64 = maxrel_cols(g32, ref), maxrel_cols(g64, ref)
    print(f"FP32 transposed level products maxrel={e32:.3e} (FP64 {e64:.3e})")
    assert e64 <= 1e-7 + 1e-12
    assert e32 <= 2e-5


def test_butterfly_adjoint_transposed_copy_matches_strided(gpu):
    # the transposed copy only changes the order of the dense sums
    L, N, B = 511, 256, 4
    maps = _dev(_maps(N, B, 750))
    pa = gpu.Plan(L, N, 1e-12, max_levels=4, store_fp32=True)
    pb = gpu.Plan(L, N, 1e-12, max_levels=4, store_fp32=True, store_transpose=True)
    assert pb.info()["device_bytes"] > pa.info()["device_bytes"]
    for prec, tol in ((sht.PREC_FP64, 1e-14), (sht.PREC_FP32, 1e-6)):
        ga = pa.adjoint(maps, path=sht.PATH_BUTTERFLY, precision=prec)
        gb = pb.adjoint(maps, path=sht.PATH_BUTTERFLY, precision=prec)
        err = float((ga - gb).abs().max() / ga.abs().max())
        print(f"prec={prec} strided vs transposed copy: {err:.3e}")
        assert err <= tol


def test_butterfly_adjoint_every_entry_written(gpu):
    L, N, B = 300, 128, 3
    maps = _dev(_maps(N, B, 760))
    p = gpu.Plan(L, N, 1e-12, max_levels=3)
    out = torch.full((p.nalm, B), complex(float("nan"), float("nan")), dtype=torch.complex128, device="cuda")
    p.adjoint(maps, out=out, path=sht.PATH_BUTTERFLY)
    assert bool(torch.isfinite(torch.view_as_real(out)).all())
    assert bool((out[:L + 1].imag == 0).all())  # m = 0 rows are real
    ref = p.adjoint(maps, path=sht.PATH_BRUTE)
    err = float((out - ref).abs().max() / ref.abs().max())
    assert err <= 1e-12 + 1e-12


def test_butterfly_adjoint_needs_eps_plan(gpu):
    p = gpu.Plan(31, 16)
    maps = _dev(_maps(16, 1, 780))
    with pytest.raises(sht.ShtError):
        p.adjoint(maps, path=sht.PATH_BUTTERFLY)


def test_butterfly_autograd_gradcheck(gpu):
    from paper_1110_4874_amd.sht import synthesis_fn
    L, N = 9, 2
    p = gpu.Plan(L, N, 1e-12, max_levels=1)
    alm = _dev(alm_gaussian(L, [6])).reshape(-1, 1).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a: synthesis_fn(p, a, path=sht.PATH_BUTTERFLY), (alm,),
                                    eps=1e-6, atol=1e-9)
