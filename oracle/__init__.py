"""CPU oracle for HEALPix spherical harmonic synthesis and its adjoint.

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It is a ctypes wrapper around
liboracle.so (plain C, oracle/oracle.c), which shares no code with the HIP
library.  Every function follows a plain definition from the Wavemoth paper
(Seljebotn, arXiv:1110.4874); the pins that tie each one to the paper and to
mathematics are in tests/test_oracle_pins.py.

Layouts: alm (nalm, B) complex128, m-major (offset(m) = m(2L+3-m)/2);
maps (B, Npix) float64 in HEALPix RING order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_l = ctypes.c_long
_pl = ctypes.POINTER(ctypes.c_long)
_ll = ctypes.c_longlong
_i = ctypes.c_int


def build() -> str:
    """Compile liboracle.so with gcc (plain C99 + OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, src, "-lm"], cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(_HERE, "oracle.c")
        inc = os.path.join(_HERE, "oracle_core.inc")
        if (not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src)
                or os.path.getmtime(_SO) < os.path.getmtime(inc)):
            build()
        L = ctypes.CDLL(_SO)
        L.oracle_ring_info.argtypes = [_l, _l, _pd, _pd, _pl, _pl, ctypes.POINTER(_ll)]
        L.oracle_pixel_ring.argtypes = [_l, _ll, _pl, _pl]
        L.oracle_plm_z.argtypes = [_i, _i, _d, _d, _pd]
        L.oracle_plm_ring.argtypes = [_i, _i, _l, _l, _pd]
        L.oracle_plm_ring_ld.argtypes = [_i, _i, _l, _l, _pd]
        for fn in (L.oracle_legendre_phase_rings, L.oracle_legendre_phase_rings_ld,
                   L.oracle_synthesis_rings, L.oracle_synthesis_rings_ld):
            fn.argtypes = [_i, _l, _i, _pd, _i, _pl, _pd]
        L.oracle_synthesis.argtypes = [_i, _l, _i, _pd, _pd]
        L.oracle_synthesis_direct.argtypes = [_i, _l, _i, _pd, _l,
                                              ctypes.POINTER(_ll), _pd]
        L.oracle_adjoint.argtypes = [_i, _l, _i, _pd, _i, _pd]
        for fn in (L.oracle_adjoint_msel, L.oracle_adjoint_msel_ld):
            fn.argtypes = [_i, _l, _i, _pd, _i, _i, ctypes.POINTER(_i), _pd]
        L.oracle_spin_z.argtypes = [_i, _i, _i, _d, _d, _pd]
        L.oracle_spin_z_ld.argtypes = [_i, _i, _i, _d, _d, _pd]
        L.oracle_spin_ring_ld.argtypes = [_i, _i, _i, _l, _l, _pd]
        for fn in (L.oracle_pol_synthesis_rings_d, L.oracle_pol_synthesis_rings_ld):
            fn.argtypes = [_i, _l, _i, _pd, _pd, _i, _pl, _pd, _pd]
        L.oracle_num_threads.restype = _i
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_pd)


def _alm_in(alm):
    alm = np.ascontiguousarray(alm, dtype=np.complex128)
    if alm.ndim == 1:
        alm = alm[:, None]
    return alm


def num_threads() -> int:
    return lib().oracle_num_threads()


def nrings(nside: int) -> int:
    return 4 * nside - 1


def ring_info(nside: int, ring: int):
    """(z, sin(theta), J, s, offset) of ring 1..4N-1 (phi_j = pi(2j+s)/J)."""
    z, st = _d(), _d()
    J, s = _l(), _l()
    off = _ll()
    lib().oracle_ring_info(nside, ring, ctypes.byref(z), ctypes.byref(st),
                           ctypes.byref(J), ctypes.byref(s), ctypes.byref(off))
    return z.value, st.value, J.value, s.value, off.value


def pixel_ring(nside: int, p: int):
    r, j = _l(), _l()
    lib().oracle_pixel_ring(nside, p, ctypes.byref(r), ctypes.byref(j))
    return r.value, j.value


def plm_z(L: int, m: int, z: float, sth: float) -> np.ndarray:
    out = np.zeros(L - m + 1)
    lib().oracle_plm_z(L, m, z, sth, _ptr(out))
    return out


def plm_ring(L: int, m: int, nside: int, ring: int, ld: bool = False) -> np.ndarray:
    out = np.zeros(L - m + 1)
    fn = lib().oracle_plm_ring_ld if ld else lib().oracle_plm_ring
    fn(L, m, nside, ring, _ptr(out))
    return out


def legendre_phase_rings(L, nside, alm, rings, ld=False) -> np.ndarray:
    """q_m(z_ring): complex (nr, L+1, B)."""
    alm = _alm_in(alm)
    B = alm.shape[1]
    rings = np.ascontiguousarray(rings, dtype=np.int64)
    out = np.zeros((len(rings), L + 1, B), dtype=np.complex128)
    fn = lib().oracle_legendre_phase_rings_ld if ld else lib().oracle_legendre_phase_rings
    fn(L, nside, B, _ptr(alm.view(np.float64)), len(rings),
       rings.ctypes.data_as(_pl), _ptr(out.view(np.float64)))
    return out


def synthesis(L, nside, alm) -> np.ndarray:
    """Full maps (B, Npix)."""
    alm = _alm_in(alm)
    B = alm.shape[1]
    out = np.zeros((B, 12 * nside * nside))
    lib().oracle_synthesis(L, nside, B, _ptr(alm.view(np.float64)), _ptr(out))
    return out


def synthesis_rings(L, nside, alm, rings, ld=False):
    """Pixel values on the listed rings: list (per ring) of (B, J) arrays."""
    alm = _alm_in(alm)
    B = alm.shape[1]
    rings = np.ascontiguousarray(rings, dtype=np.int64)
    Js = [ring_info(nside, int(r))[2] for r in rings]
    out = np.zeros((B, int(sum(Js))))
    fn = lib().oracle_synthesis_rings_ld if ld else lib().oracle_synthesis_rings
    fn(L, nside, B, _ptr(alm.view(np.float64)), len(rings),
       rings.ctypes.data_as(_pl), _ptr(out))
    res, o = [], 0
    for J in Js:
        res.append(out[:, o:o + J].copy())
        o += J
    return res


def synthesis_direct(L, nside, alm, pix) -> np.ndarray:
    """O(L^2) per pixel evaluation of the harmonic sum: (B, npix_sel)."""
    alm = _alm_in(alm)
    B = alm.shape[1]
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.zeros((B, len(pix)))
    lib().oracle_synthesis_direct(L, nside, B, _ptr(alm.view(np.float64)), len(pix),
                                  pix.ctypes.data_as(ctypes.POINTER(_ll)), _ptr(out))
    return out


def adjoint(L, nside, maps, conv: int = 0) -> np.ndarray:
    """Transpose of synthesis: (nalm, B) complex."""
    maps = np.ascontiguousarray(np.atleast_2d(maps), dtype=np.float64)
    B = maps.shape[0]
    out = np.zeros(((L + 1) * (L + 2) // 2, B), dtype=np.complex128)
    lib().oracle_adjoint(L, nside, B, _ptr(maps), conv, _ptr(out.view(np.float64)))
    return out


def adjoint_msel(L, nside, maps, ms, conv: int = 0, ld: bool = False) -> np.ndarray:
    """Adjoint for selected m: (nm, L+1, B) complex, entry [k, l-m, b] = g_lm.
    ld=True runs the same transpose in long double (rounded once)."""
    maps = np.ascontiguousarray(np.atleast_2d(maps), dtype=np.float64)
    B = maps.shape[0]
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    out = np.zeros((len(ms), L + 1, B), dtype=np.complex128)
    fn = lib().oracle_adjoint_msel_ld if ld else lib().oracle_adjoint_msel
    fn(L, nside, B, _ptr(maps), conv, len(ms),
                              ms.ctypes.data_as(ctypes.POINTER(_i)),
                              _ptr(out.view(np.float64)))
    return out


def spin_z(L: int, m: int, s: int, z: float, sth: float, ld: bool = False) -> np.ndarray:
    """Spin-weighted _s lambda_lm(theta), l = m..L (zero for l < max(m, |s|))."""
    out = np.zeros(L - m + 1)
    fn = lib().oracle_spin_z_ld if ld else lib().oracle_spin_z
    fn(L, m, s, z, sth, _ptr(out))
    return out


def spin_ring(L: int, m: int, s: int, nside: int, ring: int) -> np.ndarray:
    """Long-double _s lambda_lm at ring 1..4N-1 (exact ring geometry), l = m..L."""
    out = np.zeros(L - m + 1)
    lib().oracle_spin_ring_ld(L, m, s, nside, ring, _ptr(out))
    return out


def pol_synthesis_rings(L, nside, E, B, rings, ld=False):
    """Polarized synthesis (Q, U) from E and B modes on the listed rings:
    two lists (per ring) of (nmaps, J) arrays.  a_{+-2,lm} = -(E_lm +- i B_lm),
    Q +- iU = sum a_{+-2,lm} _{+-2}Y_lm (spin-weighted harmonics of Goldberg
    et al. 1967, Condon-Shortley phase)."""
    E, B = _alm_in(E), _alm_in(B)
    if E.shape != B.shape:
        raise ValueError("E and B must have the same shape")
    nm = E.shape[1]
    rings = np.ascontiguousarray(rings, dtype=np.int64)
    Js = [ring_info(nside, int(r))[2] for r in rings]
    oq = np.zeros((nm, int(sum(Js))))
    ou = np.zeros((nm, int(sum(Js))))
    fn = lib().oracle_pol_synthesis_rings_ld if ld else lib().oracle_pol_synthesis_rings_d
    fn(L, nside, nm, _ptr(E.view(np.float64)), _ptr(B.view(np.float64)), len(rings),
       rings.ctypes.data_as(_pl), _ptr(oq), _ptr(ou))
    rq, ru, o = [], [], 0
    for J in Js:
        rq.append(oq[:, o:o + J].copy())
        ru.append(ou[:, o:o + J].copy())
        o += J
    return rq, ru


def analysis(L, nside, maps, iterations: int = 0) -> np.ndarray:
    """Quadrature analysis of Sec. 2.2, a_lm = sum_j w_j f_j Y*_lm(j), with the
    HEALPix equal pixel weight w = 4 pi / Npix, then `iterations` Jacobi steps
    a <- a + w Y^dagger (f - Y a): (nalm, B) complex.  Composed from the
    synthesis and the dagger-convention adjoint above."""
    maps = np.ascontiguousarray(np.atleast_2d(maps), dtype=np.float64)
    w = 4.0 * np.pi / (12 * nside * nside)
    a = w * adjoint(L, nside, maps, conv=1)
    for _ in range(iterations):
        r = maps - synthesis(L, nside, a)
        a = a + w * adjoint(L, nside, r, conv=1)
    return a
