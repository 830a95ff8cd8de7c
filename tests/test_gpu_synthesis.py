"""GPU parity of synthesis against the CPU oracle (through the C ABI).

Tolerance (FP64 brute-force path): max_p |y_p - x_p| / max_p |x_p| <= 1e-12,
per map, against the FP64 oracle up to L = 511 and against the oracle's
long-double mode at L = 4095 (whose own FP64 mode is off by ~2e-11 at the
first polar rings; see the oracle pins).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1110_4874_amd.synthetic import alm_gaussian
from ring_defs import ring_direct

pytestmark = pytest.mark.gpu

TOL = 1e-12


def maxrel(y, x):
    y = np.atleast_2d(y)
    x = np.atleast_2d(x)
    return max(np.max(np.abs(y[b] - x[b])) / np.max(np.abs(x[b])) for b in range(x.shape[0]))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _oracle_q_layout(L, N, alm):
    """Oracle Legendre phase in the library's q layout (nrings, L+1, B)."""
    rings = np.arange(1, 4 * N)
    return np.ascontiguousarray(oracle.legendre_phase_rings(L, N, alm, rings))  # (nr, L+1, B)


@pytest.mark.parametrize("L,N,B", [(63, 32, 1), (40, 16, 3), (31, 16, 2), (0, 1, 1), (5, 1, 1),
                                   (70, 12, 1), (100, 24, 5)])
def test_legendre_phase_parity(gpu, L, N, B):
    alm = alm_gaussian(L, list(range(100, 100 + B)))
    p = gpu.Plan(L, N)
    q = p.legendre_phase(_dev(alm)).cpu().numpy()
    ref = _oracle_q_layout(L, N, alm)
    err = np.max(np.abs(q - ref)) / np.max(np.abs(ref))
    print(f"L={L} N={N} B={B} q maxrel={err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("L,N", [(63, 32), (40, 16), (80, 12), (29, 4), (127, 20)])
def test_ring_stage_parity(gpu, L, N):
    # feed the oracle's own q to the ring kernel: isolates phase shift, wrap and FFT
    alm = alm_gaussian(L, [7, 8])
    q = _oracle_q_layout(L, N, alm)
    p = gpu.Plan(L, N)
    f = p.ring_synthesis(_dev(q)).cpu().numpy()
    ref = oracle.synthesis(L, N, alm)
    err = maxrel(f, ref)
    print(f"L={L} N={N} ring-stage maxrel={err:.3e}")
    assert err <= TOL


# L = 2100, nside = 600: polar rings with J <= L up to ring 525 (rings 512..525
# have more bin pairs than a 512-thread workgroup), J > L from ring 526, the
# belt from 600, and their south counterparts; powers of two at 128 and 512
RINGS_2100 = [1, 2, 3, 50, 127, 128, 300, 511, 512, 518, 525, 526, 527, 599, 600, 601, 1200, 1799, 1800,
              1801, 1873, 1874, 1875, 1888, 2398, 2399]


@pytest.mark.parametrize("B", [1, 2, 3, 4])
def test_ring_stage_direct_dft_l2100(gpu, B):
    # random q straight into the ring kernel: every ring class with one, two
    # or four maps per workgroup (odd B: one), against the ring sum by its
    # definition (pinned to the oracle in test_ring_definitions.py)
    L, N = 2100, 600
    rng = np.random.default_rng(900 + B)
    nr = 4 * N - 1
    q = rng.standard_normal((nr, L + 1, B)) + 1j * rng.standard_normal((nr, L + 1, B))
    f = gpu.Plan(L, N).ring_synthesis(_dev(q)).cpu().numpy()
    worst = 0.0
    for ring in RINGS_2100:
        z, st, J, s, off = oracle.ring_info(N, ring)
        ref = ring_direct(q[ring - 1], J, s)
        worst = max(worst, float(np.max(np.abs(f[:, off:off + J] - ref)) / np.max(np.abs(ref))))
    print(f"L=2100 N=600 B={B} ring-stage maxrel={worst:.3e}")
    assert worst <= TOL


@pytest.mark.parametrize("L,N,B,seeds", [(63, 32, 1, [1]), (511, 256, 1, [2]), (47, 8, 2, [3, 4]),
                                         (0, 1, 1, [5]), (95, 48, 4, [6, 7, 8, 9]),
                                         (200, 50, 3, [10, 11, 12])])
def test_synthesis_parity_full_map(gpu, L, N, B, seeds):
    alm = alm_gaussian(L, seeds)
    p = gpu.Plan(L, N)
    f = p.synthesis(_dev(alm)).cpu().numpy()
    ref = oracle.synthesis(L, N, alm)
    err = maxrel(f, ref)
    rms = np.sqrt(np.sum((f - ref) ** 2) / np.sum(ref ** 2))
    print(f"L={L} N={N} B={B} maxrel={err:.3e} rms={rms:.3e}")
    assert err <= TOL


def test_white_spectrum_l511(gpu):
    L, N = 511, 256
    alm = alm_gaussian(L, [2], spectrum="white")
    f = gpu.Plan(L, N).synthesis(_dev(alm)).cpu().numpy()
    ref = oracle.synthesis(L, N, alm)
    assert maxrel(f, ref) <= TOL


def test_l4095_sampled_rings_vs_long_double(gpu, plan4095):
    # the benchmark's configuration: L = 4095, nside = 2048, 4 maps
    L, N, B = 4095, 2048, 4
    alm = alm_gaussian(L, [400, 401, 402, 403])
    p = plan4095
    f = p.synthesis(_dev(alm)).cpu().numpy()
    rings = [1, 2, 3, 17, 100, 255, 256, 700, 2047, 2048, 2049, 3000, 4095, 4096, 4097, 6000,
             8000, 8190, 8191]
    ref = oracle.synthesis_rings(L, N, alm, rings, ld=True)
    fmax = np.max(np.abs(f), axis=1)
    worst = 0.0
    for ring, r in zip(rings, ref):
        z, st, J, s, off = oracle.ring_info(N, ring)
        e = np.max(np.abs(f[:, off:off + J] - r), axis=1) / fmax
        worst = max(worst, float(np.max(e)))
    print(f"L=4095 sampled-ring maxrel={worst:.3e}")
    assert worst <= TOL


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_every_pixel_written_and_deterministic(gpu, threads):
    # outputs pre-filled with NaN: any pixel the ring kernel leaves unwritten,
    # or any bin it leaves uncomputed, shows up as non-finite or as a mismatch
    L, N = 300, 128  # wrapped polar rings, Bluestein and radix-2 rings, no-wrap belt
    alm = _dev(alm_gaussian(L, [1, 2, 3, 4]))
    p = gpu.Plan(L, N, ring_threads=threads)
    q = p.legendre_phase(alm)
    outs = []
    for _ in range(2):
        out = torch.full((4, p.npix), float("nan"), dtype=torch.float64, device="cuda")
        p.ring_synthesis(q, out=out)
        outs.append(out)
    assert bool(torch.isfinite(outs[0]).all())
    assert torch.equal(outs[0], outs[1])
    ref = oracle.synthesis(L, N, alm.cpu().numpy())
    assert maxrel(outs[0].cpu().numpy(), ref) <= TOL


def test_deterministic(gpu):
    L, N = 127, 64
    alm = _dev(alm_gaussian(L, [1, 2]))
    p = gpu.Plan(L, N)
    a = p.synthesis(alm)
    b = p.synthesis(alm)
    assert torch.equal(a, b)


def test_rejects_bad_buffers(gpu):
    L, N = 15, 8
    p = gpu.Plan(L, N)
    lib = gpu.load()
    import ctypes
    alm = _dev(alm_gaussian(L, [1]))
    x = p._exec(1)
    host = np.zeros(12 * N * N)
    rc = lib.sht_synthesis_ex(p._h, ctypes.byref(x), ctypes.c_void_p(alm.data_ptr()),
                              ctypes.c_void_p(host.ctypes.data))
    assert rc == gpu.SHT_EINVAL
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    x2 = p._exec(1, workspace=ws)
    out = torch.empty((1, 12 * N * N), dtype=torch.float64, device="cuda")
    rc = lib.sht_synthesis_ex(p._h, ctypes.byref(x2), ctypes.c_void_p(alm.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()))
    assert rc == gpu.SHT_ENOMEM
    with pytest.raises((gpu.ShtError, ValueError)):
        p.synthesis(alm.reshape(-1)[:-1])
    torch.cuda.synchronize()
