"""GPU parity of the interpolation form of the synthesis (Sec. 3.3, Eq. 23):
the Legendre phase at the roots of P~_N^m, then exact interpolation to the
rings, against the oracle's plain definition.  The form is exact, so the bar
is the brute-force one: max |f - f_ref| / max |f_ref| <= 1e-12 per map (at
L = 4095 against the long-double oracle on sampled rings, polar rings
included)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1110_4874_amd import sht
from paper_1110_4874_amd.synthetic import alm_gaussian

pytestmark = pytest.mark.gpu


def maxrel(y, x):
    return max(float(np.max(np.abs(y[b] - x[b])) / np.max(np.abs(x[b]))) for b in range(x.shape[0]))


@pytest.mark.parametrize("L,N,B", [(0, 1, 1), (9, 2, 2), (63, 32, 1), (255, 128, 3), (200, 64, 5), (511, 256, 2),
                                   (100, 16, 4), (40, 64, 2)])
def test_interp_synthesis_parity(gpu, L, N, B):
    alm = alm_gaussian(L, list(range(600, 600 + B)))
    p = gpu.Plan(L, N, interp=True)
    d = torch.from_numpy(alm).cuda()
    out = torch.full((B, p.npix), float("nan"), dtype=torch.float64, device="cuda")
    p.synthesis(d, out, path=sht.PATH_INTERP)
    f = out.cpu().numpy()
    assert np.isfinite(f).all()
    ref = oracle.synthesis(L, N, alm)
    err = maxrel(f, ref)
    brute = maxrel(p.synthesis(d, path=sht.PATH_BRUTE).cpu().numpy(), ref)
    print(f"L={L} N={N} B={B} interpolation maxrel={err:.3e} (brute force {brute:.3e})")
    assert err <= 1e-12


@pytest.mark.timeout(900)
def test_interp_l4095_sampled_rings(gpu):
    L, N = 4095, 2048
    sys.stderr.write("interp L=4095: plan (cache or build)\n")
    p = gpu.cached_plan(L, N, 0.0, interp=True, log=lambda s: sys.stderr.write(s + "\n"))
    alm = alm_gaussian(L, [400, 401])
    f = p.synthesis(torch.from_numpy(alm).cuda(), path=sht.PATH_INTERP).cpu().numpy()
    n_dd = p.info()["n_dd_rings"]
    rings = sorted(set([1, 2, 3, 50, 150, n_dd, n_dd + 1, 700, 2047, 2048, 3000, 4095, 4096, 6000, 8190, 8191]))
    ref = oracle.synthesis_rings(L, N, alm, rings, ld=True)
    y = np.concatenate([f[:, oracle.ring_info(N, r)[4]:oracle.ring_info(N, r)[4] + oracle.ring_info(N, r)[2]]
                        for r in rings], axis=1)
    x = np.concatenate(ref, axis=1)
    err = maxrel(y, x)
    print(f"L=4095 interpolation maxrel={err:.3e} on rings {rings}")
    assert err <= 1e-12


def test_interp_is_synthesis_only(gpu):
    p = gpu.Plan(31, 16, interp=True)
    maps = torch.zeros((1, p.npix), dtype=torch.float64, device="cuda")
    with pytest.raises(sht.ShtError):
        p.adjoint(maps, path=sht.PATH_INTERP)
    q = gpu.Plan(31, 16)
    with pytest.raises(sht.ShtError):
        q.synthesis(torch.zeros((q.nalm, 1), dtype=torch.complex128, device="cuda"), path=sht.PATH_INTERP)
