"""GPU parity of the polarized (spin-2) synthesis, the paper's Discussion's
reduction of a polarized transform to scalar transforms, against the
oracle's spin-weighted harmonics (Goldberg et al. 1967 form with the Wigner-d
recurrence, long double): Q and U on every ring at small sizes, on sampled
rings (the polar caps, both sides of the direct-recurrence threshold, the
belt and the equator) at L = 4094 with the L = 4095 plans.

Bar: max |y - x| over Q and U, divided by max |x| over Q and U, per map,
worst map <= 1e-12 on the brute-force path.  On the butterfly path the
plan's eps enters the three scalar sums, and the combination divides two of
them by sin^2(theta) >= s_pol^2 (s_pol = 0.1 sqrt((L+1)/4096), below it the
polar recurrence takes over): bar 1e-12 + eps / s_pol^2.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1110_4874_amd import sht
from paper_1110_4874_amd.synthetic import alm_gaussian

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def say(msg):
    print(msg)
    sys.stdout.flush()


def _err(Q, U, rq, ru, rings, N):
    """worst over maps of max |error| / max |reference| on the listed rings."""
    def pick(M):
        return np.concatenate([M[:, oracle.ring_info(N, r)[4]:oracle.ring_info(N, r)[4] + oracle.ring_info(N, r)[2]]
                               for r in rings], axis=1)
    yq, yu = pick(Q), pick(U)
    xq, xu = np.concatenate(rq, axis=1), np.concatenate(ru, axis=1)
    worst = 0.0
    for b in range(xq.shape[0]):
        sc = max(np.max(np.abs(xq[b])), np.max(np.abs(xu[b])))
        worst = max(worst, max(np.max(np.abs(yq[b] - xq[b])), np.max(np.abs(yu[b] - xu[b]))) / sc)
    return worst


@pytest.mark.parametrize("L,N,n,eps", [(3, 2, 1, 0.0), (8, 4, 1, 0.0), (33, 16, 2, 0.0), (128, 64, 3, 0.0),
                                       (256, 128, 2, 0.0), (128, 64, 2, 1e-12), (300, 128, 1, 1e-12),
                                       (512, 256, 1, 0.0)])
def test_pol_synthesis_all_rings(gpu, L, N, n, eps):
    p = gpu.Plan(L, N, eps, max_levels=2 if eps else -1)
    E = alm_gaussian(L - 1, list(range(700, 700 + n)))
    B = alm_gaussian(L - 1, list(range(800, 800 + n)))
    out = torch.full((2, n, p.npix), float("nan"), dtype=torch.float64, device="cuda")
    path = sht.PATH_BUTTERFLY if eps else sht.PATH_BRUTE
    p.pol_synthesis(torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda(), out, path=path)
    torch.cuda.synchronize()
    f = out.cpu().numpy()
    assert np.isfinite(f).all()
    rings = list(range(1, 4 * N))
    rq, ru = oracle.pol_synthesis_rings(L - 1, N, E, B, rings, ld=True)
    err = _err(f[0], f[1], rq, ru, rings, N)
    say(f"L={L} N={N} n={n} eps={eps} polar rings {p.info()['pol_rings']}: max rel err {err:.3e}")
    s_pol2 = 0.01 * (L + 1) / 4096.0
    assert err <= 1e-12 + eps / s_pol2


def test_pol_rejects_fp32_and_small_plans(gpu):
    p = gpu.Plan(31, 16, 1e-10, store_fp32=True)
    E = torch.zeros((31 * 32 // 2, 1), dtype=torch.complex128, device="cuda")
    with pytest.raises(sht.ShtError):
        p.pol_synthesis(E, E, path=sht.PATH_BUTTERFLY, precision=sht.PREC_FP32)
    with pytest.raises(ValueError):
        p.pol_synthesis(E[:-1], E[:-1])


def test_pol_l4094_sampled_rings(gpu, plan4095_bf):
    p, N = plan4095_bf, 2048
    n_pol = p.info()["pol_rings"]
    rings = sorted(set([1, 2, 3, 40, n_pol - 1, n_pol, n_pol + 1, n_pol + 2, 400, 1500, 2048, 3000, 4096,
                        8191 - n_pol, 8191 - n_pol + 1, 8190, 8191]))
    E = alm_gaussian(4094, [900])
    B = alm_gaussian(4094, [901])
    say(f"L=4094 polarization: oracle (long double) on {len(rings)} rings, polar rings {n_pol}")
    rq, ru = oracle.pol_synthesis_rings(4094, N, E, B, rings, ld=True)
    dE, dB = torch.from_numpy(E).cuda(), torch.from_numpy(B).cuda()
    for name, path in (("brute", sht.PATH_BRUTE), ("bf64", sht.PATH_BUTTERFLY)):
        f = p.pol_synthesis(dE, dB, path=path).cpu().numpy()
        err = _err(f[0], f[1], rq, ru, rings, N)
        say(f"L=4094 polarization {name}: max rel err {err:.3e}")
        assert err <= (1e-12 if name == "brute" else 1e-12 + 1e-12 / 0.01)
