"""GPU parity of the adjoint (transpose) of synthesis against the CPU oracle.

The adjoint is g_lm = w_m sum_k P~_l^m(z_k) sum_j y_kj e^{-i m phi_kj}
(w_0 = 1 with Im g_l0 = 0, w_m = 2 otherwise, or w_m = 1 for the Y^dagger
convention of Sec. 2.2 Eq. 7).  Tolerance: max |g - g_ref| / max |g_ref| per
map <= 1e-12 (FP64 path); at L = 4095 against the long-double oracle, since
the FP64 oracle's own polar-ring Legendre values carry ~3e-12 there.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1110_4874_amd.synthetic import alm_gaussian, gaussian_map

pytestmark = pytest.mark.gpu

TOL = 1e-12


def maxrel_cols(g, ref):
    """max over maps of max_lm |g - ref| / max_lm |ref| (alm layout (nalm, B))."""
    return max(float(np.max(np.abs(g[:, b] - ref[:, b])) / np.max(np.abs(ref[:, b])))
               for b in range(ref.shape[1]))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _maps(N, B, seed0):
    return gaussian_map(12 * N * N, [seed0 + b for b in range(B)])


def _ybar_numpy(L, N, maps, wpos):
    """Direct per-ring DFT in numpy: (nrings, L+1, B), weights applied."""
    nr = 4 * N - 1
    B = maps.shape[0]
    out = np.zeros((L + 1, nr, B), dtype=np.complex128)
    m = np.arange(L + 1)
    w = np.where(m == 0, 1.0, wpos)
    for ring in range(1, nr + 1):
        _, _, J, s, off = oracle.ring_info(N, ring)
        j = np.arange(J)
        ph = np.exp(-1j * np.pi * np.outer(m, 2 * j + s) / J)  # (L+1, J)
        out[:, ring - 1, :] = (ph @ maps[:, off:off + J].T) * w[:, None]
    out[0, :, :] = out[0, :, :].real
    return np.ascontiguousarray(np.transpose(out, (1, 0, 2)))


@pytest.mark.parametrize("L,N,B", [(0, 1, 1), (5, 1, 1), (31, 16, 2), (40, 16, 3), (70, 12, 1),
                                   (100, 24, 5), (127, 64, 2),
                                   # 600 north rings: two FP64 ring chunks, the second partial
                                   (700, 300, 4)])
def test_adjoint_parity(gpu, L, N, B):
    maps = _maps(N, B, 900)
    p = gpu.Plan(L, N)
    g = p.adjoint(_dev(maps)).cpu().numpy()
    ref = oracle.adjoint(L, N, maps)
    err = maxrel_cols(g, ref)
    print(f"L={L} N={N} B={B} adjoint maxrel={err:.3e}")
    assert err <= TOL
    # m = 0 imaginary parts are exactly zero
    assert np.all(g[:L + 1].imag == 0.0)


@pytest.mark.parametrize("conv", [0, 1])
def test_adjoint_conventions(gpu, conv):
    L, N, B = 50, 16, 2
    maps = _maps(N, B, 950)
    p = gpu.Plan(L, N)
    g = p.adjoint(_dev(maps), convention=conv).cpu().numpy()
    ref = oracle.adjoint(L, N, maps, conv=conv)
    assert maxrel_cols(g, ref) <= TOL


@pytest.mark.parametrize("L,N", [(63, 32), (80, 12), (29, 4), (127, 20)])
def test_ring_analysis_parity(gpu, L, N):
    maps = _maps(N, 2, 970)
    p = gpu.Plan(L, N)
    yb = p.ring_analysis(_dev(maps)).cpu().numpy()
    ref = _ybar_numpy(L, N, maps, 2.0)
    err = float(np.max(np.abs(yb - ref)) / np.max(np.abs(ref)))
    print(f"L={L} N={N} ring-analysis maxrel={err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("L,N", [(63, 32), (80, 12), (127, 20)])
def test_legendre_adjoint_parity(gpu, L, N):
    # numpy ybar into the adjoint Legendre kernel isolates that stage
    maps = _maps(N, 3, 980)
    p = gpu.Plan(L, N)
    g = p.legendre_adjoint(_dev(_ybar_numpy(L, N, maps, 2.0))).cpu().numpy()
    ref = oracle.adjoint(L, N, maps)
    err = maxrel_cols(g, ref)
    print(f"L={L} N={N} legendre-adjoint maxrel={err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("L,N", [(47, 16), (200, 64)])
def test_dot_product_identity(gpu, L, N):
    # <synthesis(a), y> = sum_lm Re a Re g + Im a Im g, both sides on the GPU
    B = 2
    alm = alm_gaussian(L, [31, 32])
    maps = _maps(N, B, 990)
    p = gpu.Plan(L, N)
    f = p.synthesis(_dev(alm)).cpu().numpy()
    g = p.adjoint(_dev(maps)).cpu().numpy()
    for b in range(B):
        lhs = float(np.dot(f[b], maps[b]))
        rhs = float(np.sum(alm[:, b].real * g[:, b].real + alm[:, b].imag * g[:, b].imag))
        scale = float(np.linalg.norm(f[b]) * np.linalg.norm(maps[b]))
        assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs)


def test_adjoint_deterministic_and_every_entry_written(gpu):
    L, N = 300, 128
    maps = _dev(_maps(N, 4, 1000))
    p = gpu.Plan(L, N)
    outs = []
    for _ in range(2):
        out = torch.full((p.nalm, 4), complex(float("nan"), float("nan")), dtype=torch.complex128,
                         device="cuda")
        p.adjoint(maps, out=out)
        outs.append(out)
    assert bool(torch.isfinite(torch.view_as_real(outs[0])).all())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.timeout(600)
def test_l4095_sampled_orders(gpu, plan4095):
    L, N, B = 4095, 2048, 2
    maps = _maps(N, B, 1100)
    g = plan4095.adjoint(_dev(maps)).cpu().numpy()
    ms = [0, 1, 2, 7, 64, 511, 1024, 2047, 3000, 4000, 4094, 4095]
    ref = oracle.adjoint_msel(L, N, maps, ms, ld=True)
    # scale: the largest |g_lm| of the reference over the sampled orders
    gmax = np.max(np.abs(ref), axis=(0, 1))
    worst = 0.0
    for k, m in enumerate(ms):
        o = m * (2 * L + 3 - m) // 2
        e = np.max(np.abs(g[o:o + L + 1 - m] - ref[k, :L + 1 - m]), axis=0) / gmax
        worst = max(worst, float(np.max(e)))
    print(f"L=4095 sampled-order adjoint maxrel={worst:.3e} (long-double oracle)")
    assert worst <= TOL


def test_autograd_gradcheck(gpu):
    from paper_1110_4874_amd.sht import synthesis_fn
    L, N = 6, 2
    p = gpu.Plan(L, N)
    alm = _dev(alm_gaussian(L, [5])).reshape(-1, 1).requires_grad_(True)
    # m = 0 imaginary parts do not enter synthesis; the transpose gives them zero gradient
    assert torch.autograd.gradcheck(lambda a: synthesis_fn(p, a), (alm,), eps=1e-6, atol=1e-9)
