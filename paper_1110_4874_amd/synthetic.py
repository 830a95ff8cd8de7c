"""Seeded synthetic inputs for the transform, shared by the oracle tests, the
GPU tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the
transform's arithmetic, so the oracle and the HIP path consume the same
bytes without sharing any step of the method.

Workload shape (Wavemoth paper, Sec. 4.2 and Table 2): the paper transforms
Gaussian a_lm on a HEALPix grid with Nside = L/2; the benchmark configurations
here use L = 2 Nside - 1 and a red spectrum C_l = 1/(l+1)^2 (plus a white
variant, C_l = 1, as in the paper's accuracy table).

Convention for a complex Gaussian with variance C_l: for m >= 1, Re and Im are
independent N(0, C_l/2), so E|a_lm|^2 = C_l; for m = 0 the coefficient is real,
a_l0 ~ N(0, C_l) (real-field symmetry, Sec. 2.1).  Draws are m-major with l
ascending inside each m and (Re, Im) consecutive per coefficient, from
numpy's PCG64 ``default_rng(seed)``; one seed per map.
"""
from __future__ import annotations

import numpy as np


def nalm(L: int) -> int:
    """Number of (l, m) pairs with 0 <= m <= l <= L."""
    return (L + 1) * (L + 2) // 2


def lm_index(L: int):
    """(l, m) integer arrays in the m-major order used by every layout here."""
    ls = np.concatenate([np.arange(m, L + 1) for m in range(L + 1)])
    ms = np.concatenate([np.full(L + 1 - m, m) for m in range(L + 1)])
    return ls, ms


def alm_gaussian(L: int, seeds, spectrum: str = "red") -> np.ndarray:
    """Complex128 array of shape (nalm, B): column b is drawn from seeds[b].

    spectrum: "red" (C_l = 1/(l+1)^2) or "white" (C_l = 1).
    """
    seeds = [int(s) for s in np.atleast_1d(seeds)]
    ls, ms = lm_index(L)
    if spectrum == "red":
        cl = 1.0 / (ls + 1.0) ** 2
    elif spectrum == "white":
        cl = np.ones_like(ls, dtype=np.float64)
    else:
        raise ValueError(spectrum)
    sd = np.where(ms == 0, np.sqrt(cl), np.sqrt(cl / 2.0))
    out = np.empty((nalm(L), len(seeds)), dtype=np.complex128)
    for b, seed in enumerate(seeds):
        g = np.random.default_rng(seed).standard_normal((nalm(L), 2))
        re = g[:, 0] * sd
        im = np.where(ms == 0, 0.0, g[:, 1] * sd)
        out[:, b] = re + 1j * im
    return out


def gaussian_map(npix: int, seeds, sigma=1.0) -> np.ndarray:
    """Float64 array (B, npix) of i.i.d. N(0, sigma_b^2) pixel noise."""
    seeds = [int(s) for s in np.atleast_1d(seeds)]
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (len(seeds),))
    return np.stack([np.random.default_rng(s).standard_normal(npix) * sig[b]
                     for b, s in enumerate(seeds)])


def mixed_requests(seed: int = 500, n: int = 64, lmax_choices=(127, 255, 511, 1023),
                   max_maps: int = 8):
    """Queue of synthesis requests of uneven size: list of (L, nside, B, seeds)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        L = int(rng.choice(lmax_choices))
        B = int(rng.integers(1, max_maps + 1))
        reqs.append((L, (L + 1) // 2, B, [5000 + 16 * i + b for b in range(B)]))
    return reqs
