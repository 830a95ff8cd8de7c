"""ctypes binding of libsht.so (the C ABI in include/sht.h).

Argument marshalling only: every step of the transform runs in the HIP
kernels of the library.  Torch provides device memory and streams.  If the
library has not been built this module raises instead of falling back to
anything else.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import torch  # imported first so that the library shares torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsht.so")

SHT_OK, SHT_EINVAL, SHT_ENOMEM, SHT_EDEVICE, SHT_ECORRUPT, SHT_EUNSUPPORTED, SHT_EIO = 0, -1, -2, -3, -4, -5, -6
PATH_AUTO, PATH_BRUTE, PATH_BUTTERFLY, PATH_INTERP = 0, 1, 2, 3
PREC_FP64, PREC_FP32 = 0, 1
STAGE_LEGENDRE, STAGE_RING, STAGE_RING_ADJ, STAGE_LEGENDRE_ADJ = 0, 1, 2, 3
STAGE_BF_RESIDUAL, STAGE_BF_LEVELS, NSTAGES = 4, 5, 6
ADJ_TRANSPOSE, ADJ_DAGGER = 0, 1

_c = ctypes
_lib = None


class PlanOpts(_c.Structure):
    _fields_ = [("cutoff", _c.c_double), ("dd_sin", _c.c_double), ("nthreads", _c.c_int),
                ("rings_per_lane", _c.c_int), ("ring_threads", _c.c_int), ("host_only", _c.c_int),
                ("rho", _c.c_double), ("max_levels", _c.c_int), ("chunk", _c.c_int),
                ("id_safety", _c.c_double), ("store_fp32", _c.c_int), ("batch_mib", _c.c_int),
                ("store_transpose", _c.c_int), ("interp", _c.c_int)]


class ExecOpts(_c.Structure):
    _fields_ = [("nmaps", _c.c_int), ("path", _c.c_int), ("stream", _c.c_void_p),
                ("workspace", _c.c_void_p), ("workspace_bytes", _c.c_size_t),
                ("adjoint_convention", _c.c_int), ("precision", _c.c_int),
                ("stage_events", _c.POINTER(_c.c_void_p))]


class PlanInfo(_c.Structure):
    _fields_ = [("L", _c.c_int), ("nside", _c.c_int), ("nrings", _c.c_int), ("n_dd_rings", _c.c_int),
                ("eps", _c.c_double), ("n_step", _c.c_longlong), ("n_step_exec", _c.c_longlong),
                ("n_step_dd", _c.c_longlong), ("n_step_lanes", _c.c_longlong),
                ("device_bytes", _c.c_size_t), ("build_seconds", _c.c_double),
                ("bf_built", _c.c_int), ("bf_T_entries", _c.c_longlong), ("bf_res_elems", _c.c_longlong),
                ("bf_nodes", _c.c_longlong), ("bf_units", _c.c_longlong), ("bf_res_lanes", _c.c_longlong), ("bf_res_exec", _c.c_longlong),
                ("bf_depth_hist", _c.c_longlong * 11), ("bf_build_seconds", _c.c_double),
                ("bf_nbatch", _c.c_int), ("bf_level_T", _c.c_longlong * 11),
                ("bf_level_units", _c.c_longlong * 11), ("bf_level_nodes", _c.c_longlong * 11),
                ("ip_built", _c.c_int), ("ip_nodes", _c.c_longlong), ("ip_steps", _c.c_longlong),
                ("ip_exec", _c.c_longlong), ("ip_build_seconds", _c.c_double),
                ("ip_direct", _c.c_longlong), ("pol_rings", _c.c_int)]


class Request(_c.Structure):
    _fields_ = [("plan", _c.c_void_p), ("nmaps", _c.c_int), ("alm", _c.c_void_p), ("map", _c.c_void_p)]


class BatchOpts(_c.Structure):
    _fields_ = [("stream", _c.c_void_p), ("nstreams", _c.c_int), ("path", _c.c_int), ("precision", _c.c_int),
                ("workspace", _c.c_void_p), ("workspace_bytes", _c.c_size_t), ("rings_per_lane", _c.c_int),
                ("ring_threads", _c.c_int)]


EXPORTS = {
    "sht_batch_opts_default": (None, [_c.POINTER(BatchOpts)]),
    "sht_batch_workspace_bytes": (_c.c_size_t, [_c.POINTER(Request), _c.c_int, _c.POINTER(BatchOpts)]),
    "sht_batch_execute": (_c.c_int, [_c.POINTER(Request), _c.c_int, _c.POINTER(BatchOpts)]),
    "sht_queue_workspace_bytes": (_c.c_size_t, [_c.POINTER(Request), _c.c_int, _c.POINTER(BatchOpts)]),
    "sht_batch_create": (_c.c_void_p, [_c.POINTER(Request), _c.c_int, _c.POINTER(BatchOpts)]),
    "sht_batch_run": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "sht_batch_stats": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_longlong), _c.POINTER(_c.c_int),
                                   _c.POINTER(_c.c_int)]),
    "sht_batch_free": (None, [_c.c_void_p]),
    "sht_plan_opts_default": (None, [_c.POINTER(PlanOpts)]),
    "sht_exec_opts_default": (None, [_c.POINTER(ExecOpts)]),
    "sht_plan": (_c.c_void_p, [_c.c_int, _c.c_int, _c.c_double]),
    "sht_plan_ex": (_c.c_void_p, [_c.c_int, _c.c_int, _c.c_double, _c.POINTER(PlanOpts)]),
    "sht_plan_free": (None, [_c.c_void_p]),
    "sht_plan_info": (_c.c_int, [_c.c_void_p, _c.POINTER(PlanInfo)]),
    "sht_workspace_bytes": (_c.c_size_t, [_c.c_void_p, _c.POINTER(ExecOpts)]),
    "sht_synthesis": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "sht_synthesis_ex": (_c.c_int, [_c.c_void_p, _c.POINTER(ExecOpts), _c.c_void_p, _c.c_void_p]),
    "sht_adjoint": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "sht_adjoint_ex": (_c.c_int, [_c.c_void_p, _c.POINTER(ExecOpts), _c.c_void_p, _c.c_void_p]),
    "sht_analysis_workspace_bytes": (_c.c_size_t, [_c.c_void_p, _c.POINTER(ExecOpts)]),
    "sht_analysis_ex": (_c.c_int, [_c.c_void_p, _c.POINTER(ExecOpts), _c.c_void_p, _c.c_void_p, _c.c_int]),
    "sht_debug_ring_analysis": (_c.c_int, [_c.c_void_p, _c.POINTER(ExecOpts), _c.c_void_p, _c.c_void_p]),
    "sht_debug_legendre_adjoint": (_c.c_int, [_c.c_void_p, _c.POINTER(ExecOpts), _c.c_void_p, _c.c_void_p]),
    "sht_last_error": (_c.c_char_p, []),
    "sht_last_status": (_c.c_int, []),
    "sht_noalloc_scratch_bytes": (_c.c_size_t, []),
    "sht_synthesis_noalloc": (_c.c_int, [_c.c_void_p, _c.POINTER(ExecOpts), _c.c_void_p, _c.c_void_p]),
    "sht_sync_status": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "sht_plan_save": (_c.c_int, [_c.c_void_p, _c.c_char_p]),
    "sht_plan_load": (_c.c_void_p, [_c.c_char_p]),
    "sht_plan_load_ex": (_c.c_void_p, [_c.c_char_p, _c.POINTER(PlanOpts)]),
    "sht_debug_legendre_phase": (_c.c_int, [_c.c_void_p, _c.POINTER(ExecOpts), _c.c_void_p, _c.c_void_p]),
    "sht_debug_ring_synthesis": (_c.c_int, [_c.c_void_p, _c.POINTER(ExecOpts), _c.c_void_p, _c.c_void_p]),
    "sht_debug_coef": (_c.c_int, [_c.c_void_p, _c.c_int, _c.POINTER(_c.c_double)]),
    "sht_debug_interp_decomp": (_c.c_int, [_c.c_void_p, _c.c_int, _c.c_int, _c.c_double,
                                           _c.POINTER(_c.c_int), _c.c_void_p, _c.c_void_p]),
    "sht_debug_butterfly_apply": (_c.c_int, [_c.c_void_p, _c.c_int, _c.c_int, _c.c_void_p, _c.c_void_p]),
    "sht_debug_butterfly_depth": (_c.c_int, [_c.c_void_p, _c.c_int, _c.c_int]),
    "sht_debug_interp_apply": (_c.c_int, [_c.c_void_p, _c.c_int, _c.c_int, _c.c_void_p, _c.c_void_p]),
    "sht_pol_workspace_bytes": (_c.c_size_t, [_c.c_void_p, _c.POINTER(ExecOpts)]),
    "sht_pol_synthesis": (_c.c_int, [_c.c_void_p, _c.POINTER(ExecOpts), _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "sht_debug_pol_column": (_c.c_int, [_c.c_void_p, _c.c_int, _c.c_int, _c.c_int, _c.c_void_p]),
    "sht_debug_start": (_c.c_int, [_c.c_void_p, _c.c_int, _c.c_int, _c.c_int, _c.POINTER(_c.c_int),
                                   _c.POINTER(_c.c_double)]),
}


class ShtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sht error {code}: {msg}")
        self.code = code


def load():
    """Load libsht.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1110_4874_amd.build`")
        lib = _c.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc):
    if rc != SHT_OK:
        raise ShtError(rc, load().sht_last_error().decode())


def interp_decomp(A, tol):
    """Host interpolative decomposition as the butterfly precompute takes it
    (private test entry point).  A: (r, c) float64.  Returns (k, piv, T)."""
    import numpy as np
    A = np.asarray(A, dtype=np.float64)
    r, c = A.shape
    Af = np.asfortranarray(A)
    k = _c.c_int(0)
    piv = np.zeros(c, dtype=np.int32)
    T = np.zeros(c * c, dtype=np.float64)
    _check(load().sht_debug_interp_decomp(Af.ctypes.data_as(_c.c_void_p), r, c, float(tol), _c.byref(k),
                                          piv.ctypes.data_as(_c.c_void_p), T.ctypes.data_as(_c.c_void_p)))
    kk = k.value
    return kk, piv, T[:kk * (c - kk)].reshape(kk, c - kk)


def nalm(L):
    return (L + 1) * (L + 2) // 2


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return _c.c_void_p(s.cuda_stream)


def _on(stream):
    """Context in which a call's temporaries (outputs, workspace, contiguous
    copies) are allocated and copied on the stream its kernels run on, so the
    caching allocator never hands their memory to other work while the
    kernels may still use it."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


class Plan:
    """A transform plan for band limit L on a HEALPix grid of resolution nside."""

    def __init__(self, L, nside, eps=0.0, *, cutoff=None, dd_sin=None, nthreads=0, rings_per_lane=0,
                 ring_threads=0, host_only=False, rho=0.0, max_levels=-1, chunk=0, id_safety=0.0,
                 store_fp32=False, batch_mib=0, store_transpose=False, interp=False):
        lib = load()
        o = PlanOpts()
        lib.sht_plan_opts_default(_c.byref(o))
        o.rho = float(rho)
        o.max_levels = int(max_levels)
        o.chunk = int(chunk)
        o.id_safety = float(id_safety)
        o.store_fp32 = 1 if store_fp32 else 0
        o.batch_mib = int(batch_mib)
        o.store_transpose = 1 if store_transpose else 0
        o.interp = 1 if interp else 0
        if cutoff is not None:
            o.cutoff = cutoff
        if dd_sin is not None:
            o.dd_sin = dd_sin
        o.nthreads = nthreads
        o.rings_per_lane = rings_per_lane
        o.ring_threads = ring_threads
        o.host_only = 1 if host_only else 0
        if not host_only:
            torch.cuda.init()
        h = lib.sht_plan_ex(int(L), int(nside), float(eps), _c.byref(o))
        if not h:
            raise ShtError(lib.sht_last_status(), lib.sht_last_error().decode())
        self._adopt(h, host_only)

    def _adopt(self, h, host_only):
        self._h = _c.c_void_p(h)
        inf = self.info()
        self.L, self.nside, self.eps = int(inf["L"]), int(inf["nside"]), float(inf["eps"])
        self.nrings = 4 * self.nside - 1
        self.npix = 12 * self.nside * self.nside
        self.nalm = nalm(self.L)
        self.host_only = bool(host_only)

    @classmethod
    def load(cls, path, *, host_only=False, store_fp32=False, store_transpose=False, nthreads=0):
        """A plan from a file written by save() (sht_plan_load_ex): the saved
        operator, on cuda's current device unless host_only."""
        lib = load()
        o = PlanOpts()
        lib.sht_plan_opts_default(_c.byref(o))
        o.host_only = 1 if host_only else 0
        o.store_fp32 = 1 if store_fp32 else 0
        o.store_transpose = 1 if store_transpose else 0
        o.nthreads = int(nthreads)
        if not host_only:
            torch.cuda.init()
        h = lib.sht_plan_load_ex(os.fsencode(path), _c.byref(o))
        if not h:
            raise ShtError(lib.sht_last_status(), lib.sht_last_error().decode())
        self = cls.__new__(cls)
        self._adopt(h, host_only)
        return self

    def save(self, path):
        """Write the plan to `path` (sht_plan_save)."""
        _check(load().sht_plan_save(self._h, os.fsencode(path)))

    def sync(self, stream=None):
        """Wait for the work queued on `stream` and raise ShtError if the
        device reported an error for it (sht_sync_status)."""
        _check(load().sht_sync_status(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None):
            load().sht_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        inf = PlanInfo()
        _check(load().sht_plan_info(self._h, _c.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in PlanInfo._fields_}
        d["bf_depth_hist"] = list(inf.bf_depth_hist)
        d["bf_level_T"] = list(inf.bf_level_T)
        d["bf_level_units"] = list(inf.bf_level_units)
        d["bf_level_nodes"] = list(inf.bf_level_nodes)
        return d

    def butterfly_apply_host(self, m, t, x):
        """Host evaluation of Lambda^T x for (m, parity t) from the compressed
        records (private test entry point); x: numpy float64 of length n_t."""
        import numpy as np
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(2 * self.nside, dtype=np.float64)
        _check(load().sht_debug_butterfly_apply(self._h, int(m), int(t), x.ctypes.data_as(_c.c_void_p),
                                                y.ctypes.data_as(_c.c_void_p)))
        return y

    def interp_apply_host(self, m, t, x):
        """Host evaluation of q^t_m on the north rings through the plan's
        interpolation form (private test entry point)."""
        import numpy as np
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(2 * self.nside, dtype=np.float64)
        _check(load().sht_debug_interp_apply(self._h, int(m), int(t), x.ctypes.data_as(_c.c_void_p),
                                             y.ctypes.data_as(_c.c_void_p)))
        return y

    def pol_column_host(self, m, s, k):
        """_s lambda_lm, l = m .. L-1, at polar ring k by the host form of the
        polarized synthesis' polar recurrence (private test entry point)."""
        import numpy as np
        y = np.zeros(self.L - m, dtype=np.float64)
        _check(load().sht_debug_pol_column(self._h, int(m), int(s), int(k), y.ctypes.data_as(_c.c_void_p)))
        return y

    def butterfly_depth(self, m, t):
        return int(load().sht_debug_butterfly_depth(self._h, int(m), int(t)))

    # ---- execution ----------------------------------------------------
    def _exec(self, nmaps, path=PATH_AUTO, stream=None, workspace=None, events=None, convention=ADJ_TRANSPOSE,
              precision=PREC_FP64):
        x = ExecOpts()
        load().sht_exec_opts_default(_c.byref(x))
        x.nmaps = int(nmaps)
        x.path = int(path)
        x.precision = int(precision)
        x.adjoint_convention = int(convention)
        x.stream = _stream_handle(stream)
        if workspace is not None:
            x.workspace = _c.c_void_p(workspace.data_ptr())
            x.workspace_bytes = workspace.numel() * workspace.element_size()
        if events is not None:
            # events: list of 2*NSTAGES torch.cuda.Event (already recorded once) or None
            arr = (_c.c_void_p * (2 * NSTAGES))()
            for i, ev in enumerate(events):
                arr[i] = _c.c_void_p(ev.cuda_event) if ev is not None else None
            x.stage_events = arr
            self._keep = arr
        return x

    def workspace_bytes(self, nmaps=1, path=PATH_AUTO, precision=PREC_FP64):
        x = self._exec(nmaps, path=path, precision=precision)
        return int(load().sht_workspace_bytes(self._h, _c.byref(x)))

    def workspace(self, nmaps=1, device="cuda", path=PATH_AUTO, precision=PREC_FP64):
        return torch.empty(self.workspace_bytes(nmaps, path, precision), dtype=torch.uint8, device=device)

    def _alm_arg(self, alm):
        if alm.dtype != torch.complex128 or not alm.is_cuda:
            raise TypeError("alm must be a complex128 CUDA tensor")
        a = alm if alm.dim() == 2 else alm.reshape(-1, 1)
        if a.shape[0] != self.nalm:
            raise ValueError(f"alm has {a.shape[0]} rows, expected nalm = {self.nalm}")
        return a.contiguous()

    def synthesis(self, alm, out=None, *, path=PATH_AUTO, stream=None, workspace=None, events=None,
                  precision=PREC_FP64):
        """maps (B, Npix) float64 from alm (nalm, B) or (nalm,) complex128."""
        with _on(stream):
            a = self._alm_arg(alm)
            B = a.shape[1]
            if out is None:
                out = torch.empty((B, self.npix), dtype=torch.float64, device=a.device)
            if workspace is None:
                workspace = self.workspace(B, a.device, path, precision)
            x = self._exec(B, path, stream, workspace, events, precision=precision)
            _check(load().sht_synthesis_ex(self._h, _c.byref(x), _c.c_void_p(a.data_ptr()),
                                           _c.c_void_p(out.data_ptr())))
            return out

    def pol_workspace_bytes(self, nmaps=1, path=PATH_AUTO, precision=PREC_FP64):
        x = self._exec(nmaps, path=path, precision=precision)
        return int(load().sht_pol_workspace_bytes(self._h, _c.byref(x)))

    def pol_synthesis(self, E, B, out=None, *, path=PATH_AUTO, stream=None, workspace=None, events=None,
                      precision=PREC_FP64):
        """Polarized synthesis: (2, n, Npix) float64 Q and U maps from E and B
        modes, each (nalm(L-1), n) or (nalm(L-1),) complex128 (band limit
        L - 1 of this plan)."""
        with _on(stream):
            nal = self.L * (self.L + 1) // 2
            ea, ba = [], []
            for name, A, acc in (("E", E, ea), ("B", B, ba)):
                if A.dtype != torch.complex128 or not A.is_cuda:
                    raise TypeError(f"{name} must be a complex128 CUDA tensor")
                a = A if A.dim() == 2 else A.reshape(-1, 1)
                if a.shape[0] != nal:
                    raise ValueError(f"{name} has {a.shape[0]} rows, expected nalm(L-1) = {nal}")
                acc.append(a.contiguous())
            e, b = ea[0], ba[0]
            if e.shape != b.shape:
                raise ValueError("E and B must have the same shape")
            n = e.shape[1]
            if out is None:
                out = torch.empty((2, n, self.npix), dtype=torch.float64, device=e.device)
            if workspace is None:
                workspace = torch.empty(self.pol_workspace_bytes(n, path, precision), dtype=torch.uint8,
                                        device=e.device)
            x = self._exec(n, path, stream, workspace, events, precision=precision)
            _check(load().sht_pol_synthesis(self._h, _c.byref(x), _c.c_void_p(e.data_ptr()),
                                            _c.c_void_p(b.data_ptr()), _c.c_void_p(out.data_ptr())))
            return out

    def _map_arg(self, maps):
        if maps.dtype != torch.float64 or not maps.is_cuda:
            raise TypeError("maps must be a float64 CUDA tensor")
        m = maps if maps.dim() == 2 else maps.reshape(1, -1)
        if m.shape[1] != self.npix:
            raise ValueError(f"maps have {m.shape[1]} pixels, expected {self.npix}")
        return m.contiguous()

    def adjoint(self, maps, out=None, *, path=PATH_AUTO, stream=None, workspace=None, events=None,
                convention=ADJ_TRANSPOSE, precision=PREC_FP64):
        """alm (nalm, B) complex128 = A^T maps, maps (B, Npix) or (Npix,) float64.

        path and precision select the Legendre part as for synthesis (the
        butterfly adjoint is the exact transpose of that plan's compressed
        synthesis)."""
        with _on(stream):
            m = self._map_arg(maps)
            B = m.shape[0]
            if out is None:
                out = torch.empty((self.nalm, B), dtype=torch.complex128, device=m.device)
            if workspace is None:
                workspace = self.workspace(B, m.device, path, precision)
            x = self._exec(B, path, stream, workspace, events, convention, precision)
            _check(load().sht_adjoint_ex(self._h, _c.byref(x), _c.c_void_p(m.data_ptr()),
                                         _c.c_void_p(out.data_ptr())))
            return out

    def analysis_workspace(self, nmaps=1, device="cuda", path=PATH_AUTO, precision=PREC_FP64):
        x = self._exec(nmaps, path=path, precision=precision)
        nbytes = int(load().sht_analysis_workspace_bytes(self._h, _c.byref(x)))
        return torch.empty(nbytes, dtype=torch.uint8, device=device)

    def analysis(self, maps, out=None, *, iterations=0, path=PATH_AUTO, stream=None, workspace=None,
                 precision=PREC_FP64):
        """alm (nalm, B) complex128 from maps (B, Npix) or (Npix,) float64: the
        quadrature rule with weight 4 pi / Npix, then `iterations` Jacobi steps
        a <- a + w Y^dagger (maps - Y a)."""
        with _on(stream):
            m = self._map_arg(maps)
            B = m.shape[0]
            if out is None:
                out = torch.empty((self.nalm, B), dtype=torch.complex128, device=m.device)
            if workspace is None:
                workspace = self.analysis_workspace(B, m.device, path, precision)
            x = self._exec(B, path, stream, workspace, None, ADJ_DAGGER, precision)
            _check(load().sht_analysis_ex(self._h, _c.byref(x), _c.c_void_p(m.data_ptr()),
                                          _c.c_void_p(out.data_ptr()), int(iterations)))
            return out

    def ring_analysis(self, maps, *, stream=None, convention=ADJ_TRANSPOSE):
        """ybar (nrings, L+1, B) complex128 (private test entry point)."""
        with _on(stream):
            m = self._map_arg(maps)
            B = m.shape[0]
            yb = torch.empty((self.nrings, self.L + 1, B), dtype=torch.complex128, device=m.device)
            x = self._exec(B, stream=stream, convention=convention)
            _check(load().sht_debug_ring_analysis(self._h, _c.byref(x), _c.c_void_p(m.data_ptr()),
                                                  _c.c_void_p(yb.data_ptr())))
            return yb

    def legendre_adjoint(self, ybar, *, stream=None):
        """alm (nalm, B) from ybar (nrings, L+1, B) (private test entry point)."""
        with _on(stream):
            yb = ybar.contiguous()
            B = yb.shape[2]
            out = torch.empty((self.nalm, B), dtype=torch.complex128, device=yb.device)
            x = self._exec(B, stream=stream)
            _check(load().sht_debug_legendre_adjoint(self._h, _c.byref(x), _c.c_void_p(yb.data_ptr()),
                                                     _c.c_void_p(out.data_ptr())))
            return out

    def legendre_phase(self, alm, *, stream=None):
        """q (nrings, L+1, B) complex128 (private test entry point)."""
        with _on(stream):
            a = self._alm_arg(alm)
            B = a.shape[1]
            q = torch.empty((self.nrings, self.L + 1, B), dtype=torch.complex128, device=a.device)
            x = self._exec(B, stream=stream)
            _check(load().sht_debug_legendre_phase(self._h, _c.byref(x), _c.c_void_p(a.data_ptr()),
                                                   _c.c_void_p(q.data_ptr())))
            return q

    def ring_synthesis(self, q, out=None, *, stream=None):
        """maps (B, Npix) from q (nrings, L+1, B) complex128 (private test entry point)."""
        with _on(stream):
            q = q.contiguous()
            B = q.shape[2]
            if out is None:
                out = torch.empty((B, self.npix), dtype=torch.float64, device=q.device)
            x = self._exec(B, stream=stream)
            _check(load().sht_debug_ring_synthesis(self._h, _c.byref(x), _c.c_void_p(q.data_ptr()),
                                                   _c.c_void_p(out.data_ptr())))
            return out

    # ---- host tables ----------------------------------------------------
    def coef(self, m):
        buf = (_c.c_double * (3 * (self.L - m + 1)))()
        _check(load().sht_debug_coef(self._h, int(m), buf))
        import numpy as np
        return np.frombuffer(buf, dtype=np.float64).reshape(-1, 3).copy()

    def start(self, m, t, k):
        idx = _c.c_int()
        vals = (_c.c_double * 2)()
        _check(load().sht_debug_start(self._h, int(m), int(t), int(k), _c.byref(idx), vals))
        return idx.value, (vals[0], vals[1])


def cached_plan(L, nside, eps=0.0, *, cache_dir=None, store_fp32=False, store_transpose=False,
                log=None, **opts):
    """A plan for (L, nside, eps, opts) from a plan file in `cache_dir`
    (default: $SHT_PLAN_CACHE, else ~/.cache/wavemoth_hip), or built and
    saved there when there is room.  A file that fails its integrity checks
    is rebuilt.  The store flags are device-side copies made at load, so one
    file serves every combination of them."""
    import shutil
    d = cache_dir or os.environ.get("SHT_PLAN_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                                       "wavemoth_hip")
    key = "_".join(f"{k}{opts[k]}" for k in sorted(opts) if k not in ("nthreads",))
    path = os.path.join(d, f"L{L}_n{nside}_eps{eps:g}" + (f"_{key}" if key else "") + ".plan")
    say = log or (lambda msg: None)
    if os.path.exists(path):
        try:
            p = Plan.load(path, store_fp32=store_fp32, store_transpose=store_transpose,
                          nthreads=opts.get("nthreads", 0))
            say(f"plan loaded from {path}")
            return p
        except ShtError as e:
            say(f"plan file {path} refused ({e}); rebuilding")
            os.remove(path)
    p = Plan(L, nside, eps, store_fp32=store_fp32, store_transpose=store_transpose, **opts)
    inf = p.info()
    need = 8 * inf["bf_T_entries"] + 24 * inf["bf_res_lanes"] + 64 * nalm(L) + (1 << 30)
    try:
        os.makedirs(d, exist_ok=True)
        if shutil.disk_usage(d).free > 2 * need + (20 << 30):
            p.save(path)
            say(f"plan saved to {path}")
    except (OSError, ShtError) as e:
        say(f"plan not cached ({e})")
    return p


class Batch:
    """A fixed list of synthesis requests (plan, alm, out) run by one
    sht_batch_execute call: longest first over a few internal streams."""

    def __init__(self, requests, *, nstreams=4, path=PATH_AUTO, precision=PREC_FP64):
        lib = load()
        self.items = []
        for plan, alm, out in requests:
            a = plan._alm_arg(alm)
            if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
                raise TypeError("out must be a contiguous float64 CUDA tensor")
            if out.numel() != a.shape[1] * plan.npix:
                raise ValueError("out has the wrong size")
            self.items.append((plan, a, out))
        n = len(self.items)
        self._reqs = (Request * max(n, 1))()
        for i, (plan, a, out) in enumerate(self.items):
            self._reqs[i].plan = plan._h
            self._reqs[i].nmaps = a.shape[1]
            self._reqs[i].alm = _c.c_void_p(a.data_ptr())
            self._reqs[i].map = _c.c_void_p(out.data_ptr())
        self.n = n
        o = BatchOpts()
        lib.sht_batch_opts_default(_c.byref(o))
        o.nstreams, o.path, o.precision = int(nstreams), int(path), int(precision)
        self._opts = o
        nb = int(lib.sht_batch_workspace_bytes(self._reqs, n, _c.byref(o)))
        dev = self.items[0][1].device if n else torch.device("cuda")
        self.workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        o.workspace = _c.c_void_p(self.workspace.data_ptr())
        o.workspace_bytes = self.workspace.numel()

    def run(self, stream=None):
        self._opts.stream = _stream_handle(stream)
        _check(load().sht_batch_execute(self._reqs, self.n, _c.byref(self._opts)))


class QueueBatch:
    """A fixed list of synthesis requests (plan, alm, out) prepared once as a
    work-queue batch (sht_batch_create): each run() is one persistent
    Legendre launch plus one ring launch per ring size class on the brute
    force path; on the butterfly path one launch per butterfly stage and
    map-group width over every request, then the ring launches.  Nothing is
    allocated in run(); runs can be captured into a graph.
    The inputs, outputs and the workspace held here must stay alive and must
    not be reused while the batch exists."""

    def __init__(self, requests, *, path=None, precision=None, rings_per_lane=0, ring_threads=0):
        lib = load()
        path = PATH_BRUTE if path is None else path
        precision = PREC_FP64 if precision is None else precision
        self.items = []
        for plan, alm, out in requests:
            a = plan._alm_arg(alm)
            if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
                raise TypeError("out must be a contiguous float64 CUDA tensor")
            if out.numel() != a.shape[1] * plan.npix:
                raise ValueError("out has the wrong size")
            self.items.append((plan, a, out))
        n = len(self.items)
        self._reqs = (Request * max(n, 1))()
        for i, (plan, a, out) in enumerate(self.items):
            self._reqs[i].plan = plan._h
            self._reqs[i].nmaps = a.shape[1]
            self._reqs[i].alm = _c.c_void_p(a.data_ptr())
            self._reqs[i].map = _c.c_void_p(out.data_ptr())
        o = BatchOpts()
        lib.sht_batch_opts_default(_c.byref(o))
        o.path, o.precision = int(path), int(precision)
        o.rings_per_lane, o.ring_threads = int(rings_per_lane), int(ring_threads)
        nb = int(lib.sht_queue_workspace_bytes(self._reqs, n, _c.byref(o)))
        if nb == 0:
            raise ShtError(lib.sht_last_status(), lib.sht_last_error().decode())
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.items[0][1].device)
        o.workspace = _c.c_void_p(self.workspace.data_ptr())
        o.workspace_bytes = nb
        h = lib.sht_batch_create(self._reqs, n, _c.byref(o))
        if not h:
            raise ShtError(lib.sht_last_status(), lib.sht_last_error().decode())
        self._h = _c.c_void_p(h)

    def run(self, stream=None):
        _check(load().sht_batch_run(self._h, _stream_handle(stream)))

    def stats(self):
        items, launches, waves = _c.c_longlong(0), _c.c_int(0), _c.c_int(0)
        _check(load().sht_batch_stats(self._h, _c.byref(items), _c.byref(launches), _c.byref(waves)))
        return {"items": items.value, "launches": launches.value, "waves": waves.value}

    def close(self):
        if getattr(self, "_h", None):
            load().sht_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Synthesis(torch.autograd.Function):
    """maps = synthesis(alm) with the hand-written transpose as its backward.

    For a real loss, torch's gradient of a complex leaf is dL/dRe + i dL/dIm,
    which is the adjoint under the real inner product (convention
    ADJ_TRANSPOSE); Im a_l0 does not enter synthesis and gets zero gradient.
    """

    @staticmethod
    def forward(ctx, plan, alm, path, precision):
        ctx.plan = plan
        ctx.shape = alm.shape
        ctx.path = path
        ctx.precision = precision
        return plan.synthesis(alm.detach(), path=path, precision=precision)

    @staticmethod
    def backward(ctx, grad_maps):
        g = ctx.plan.adjoint(grad_maps.contiguous(), convention=ADJ_TRANSPOSE, path=ctx.path,
                             precision=ctx.precision)
        return None, g.reshape(ctx.shape), None, None


def synthesis_fn(plan, alm, *, path=PATH_AUTO, precision=PREC_FP64):
    """Differentiable synthesis: alm (nalm, B) or (nalm,) complex128 -> maps.

    The backward runs the adjoint with the same path and precision, so on a
    butterfly plan the gradient is exact for the compressed operator."""
    return _Synthesis.apply(plan, alm, path, precision)
