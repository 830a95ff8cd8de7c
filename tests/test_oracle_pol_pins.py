"""Pins of the oracle's polarized (spin-2) synthesis.

The paper's Discussion reduces the transform of a polarized map to scalar
transforms, citing other work; the oracle evaluates the spin-weighted
harmonics themselves instead (Wigner-d recurrence in l from Goldberg's
closed form at the first l), so that it shares nothing with that reduction.
Each test ties the oracle to something outside it:

  spin columns      -> Goldberg et al. (1967) explicit finite sum in 40-digit
                       arithmetic (mpmath), s = 0, +2, -2, l <= 12
  s = 0             -> the scalar P~ of the scalar oracle (Sec. 2.1)
  normalisation     -> Gauss-Legendre orthonormality for l <= 40
  hemispheres       -> _s lambda_lm(pi - theta) = (-1)^(l+m) _{-s} lambda_lm(theta)
  E/B conventions,  -> textbook closed forms of the l = 2 harmonics,
  ring DFT            _2Y_20 = sqrt(15/(32 pi)) sin^2(theta), etc.
  precision modes   -> FP64 and long double agree at L = 96
"""
import math

import numpy as np
import pytest

import oracle
from paper_1110_4874_amd.synthetic import alm_gaussian, nalm


def _goldberg(s, l, m, th, mp):
    th = mp.mpf(th)
    if l < max(abs(m), abs(s)):
        return mp.mpf(0)
    pre = (-1) ** m * mp.sqrt(mp.factorial(l + m) * mp.factorial(l - m) * (2 * l + 1)
                              / (4 * mp.pi * mp.factorial(l + s) * mp.factorial(l - s)))
    tot = mp.mpf(0)
    for r in range(0, l - s + 1):
        k = r + s - m
        if k < 0 or k > l + s:
            continue
        tot += mp.binomial(l - s, r) * mp.binomial(l + s, k) * (-1) ** (l - r - s) * mp.cot(th / 2) ** (2 * r + s - m)
    return pre * mp.sin(th / 2) ** (2 * l) * tot


@pytest.mark.parametrize("ld", [False, True])
def test_spin_columns_match_goldberg(ld):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    worst = 0.0
    for th in (0.01, 0.3, 1.1, 2.0, 2.9, 3.13):
        z, st = math.cos(th), math.sin(th)
        for s in (2, -2, 0):
            for m in range(0, 13):
                col = oracle.spin_z(12, m, s, z, st, ld=ld)
                for l in range(m, 13):
                    worst = max(worst, abs(col[l - m] - float(_goldberg(s, l, m, th, mp))))
    assert worst < 5e-14


def test_spin_zero_is_the_scalar_function():
    for th in (0.05, 0.7, 1.5, 2.6):
        z, st = math.cos(th), math.sin(th)
        for m in (0, 1, 5, 40, 63):
            a = oracle.spin_z(64, m, 0, z, st)
            b = oracle.plm_z(64, m, z, st)
            assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("s", [2, -2])
def test_spin_orthonormality(s):
    L = 40
    x, w = np.polynomial.legendre.leggauss(64)
    for m in (0, 1, 2, 7, 30):
        cols = np.array([oracle.spin_z(L, m, s, xi, math.sqrt(1 - xi * xi)) for xi in x])  # (nodes, l)
        G = 2 * np.pi * (cols * w[:, None]).T @ cols
        lo = max(m, 2) - m
        G = G[lo:, lo:]
        assert np.max(np.abs(G - np.eye(G.shape[0]))) < 1e-13


def test_spin_hemisphere_symmetry():
    L = 200
    for th in (0.02, 0.4, 1.2):
        z, st = math.cos(th), math.sin(th)
        for m in (0, 1, 2, 3, 50, 150):
            for s in (2, -2):
                a = oracle.spin_z(L, m, s, -z, st)
                b = oracle.spin_z(L, m, -s, z, st)
                sign = np.array([(-1) ** (l + m) for l in range(m, L + 1)])
                assert np.max(np.abs(a - sign * b)) < 1e-12


def _single(L, l, m, val):
    a = np.zeros((nalm(L), 1), dtype=np.complex128)
    a[m * (2 * L + 3 - m) // 2 + l - m, 0] = val
    return a


def test_pol_closed_forms_l2():
    """E_20 = 1: Q = -sqrt(15/(32 pi)) sin^2(theta), U = 0; B_20 = 1: the
    same in U.  E_22 = 1: Q = -2 F1_22 cos(2 phi), U = -2 F2_22 sin(2 phi)
    with F1_22 = sqrt(5/(4 pi)) (sin^4(theta/2) + cos^4(theta/2))/2 and
    F2_22 = -sqrt(5/(4 pi)) cos(theta)/2."""
    L, N = 6, 4
    rings = list(range(1, 4 * N))
    zero = np.zeros((nalm(L), 1), dtype=np.complex128)
    c20 = math.sqrt(15 / (32 * math.pi))
    Q, U = oracle.pol_synthesis_rings(L, N, _single(L, 2, 0, 1.0), zero, rings)
    Qb, Ub = oracle.pol_synthesis_rings(L, N, zero, _single(L, 2, 0, 1.0), rings)
    Q2, U2 = oracle.pol_synthesis_rings(L, N, _single(L, 2, 2, 1.0), zero, rings)
    for k, r in enumerate(rings):
        z, st, J, s, _ = oracle.ring_info(N, r)
        phi = np.pi * (2 * np.arange(J) + s) / J
        assert np.allclose(Q[k][0], -c20 * st * st, atol=1e-14, rtol=0)
        assert np.allclose(U[k][0], 0.0, atol=1e-14)
        assert np.allclose(Ub[k][0], -c20 * st * st, atol=1e-14, rtol=0)
        assert np.allclose(Qb[k][0], 0.0, atol=1e-14)
        th = math.acos(z)
        f1 = math.sqrt(5 / (4 * math.pi)) * (math.sin(th / 2) ** 4 + math.cos(th / 2) ** 4) / 2
        f2 = -math.sqrt(5 / (4 * math.pi)) * z / 2
        assert np.allclose(Q2[k][0], -2 * f1 * np.cos(2 * phi), atol=1e-14, rtol=0)
        assert np.allclose(U2[k][0], -2 * f2 * np.sin(2 * phi), atol=1e-14, rtol=0)


def test_pol_long_double_matches_fp64():
    L, N = 96, 48
    E = alm_gaussian(L, [11, 12])
    B = alm_gaussian(L, [13, 14])
    rings = [1, 2, 17, 48, 95, 96, 150, 190, 191]
    qd, ud = oracle.pol_synthesis_rings(L, N, E, B, rings)
    ql, ul = oracle.pol_synthesis_rings(L, N, E, B, rings, ld=True)
    scale = max(np.max(np.abs(np.concatenate(ql, axis=1))), np.max(np.abs(np.concatenate(ul, axis=1))))
    for a, b in zip(qd + ud, ql + ul):
        assert np.max(np.abs(a - b)) / scale < 1e-13
