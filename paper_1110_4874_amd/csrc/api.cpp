// C ABI entry points (include/sht.h): argument checking, workspace
// management and the launch sequence of each transform.
#include <chrono>
#include <cstring>
#include <new>

#include "internal.h"

namespace sht {
const char *last_error();
int last_status();
size_t synth_ws_bytes_impl(const sht_plan_s *p, int nmaps, int path, int precision);
}

using namespace sht;

namespace {

struct DeviceGuard {  // make the plan's device current for the call
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace sht {
// The pointer must be device memory of `dev` with at least `bytes` bytes
// left in its allocation; checked before any kernel may touch it.
int check_dev_ptr(const void *ptr, size_t bytes, int dev, const char *name) {
    if (!ptr) return fail(SHT_EINVAL, std::string(name) + " is NULL");
    hipPointerAttribute_t at;
    std::memset(&at, 0, sizeof(at));
    if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SHT_EINVAL, std::string(name) + " is not a device pointer");
    }
    if (at.type != hipMemoryTypeDevice)
        return fail(SHT_EINVAL, std::string(name) + " is not device memory");
    if (at.device != dev)
        return fail(SHT_EINVAL, std::string(name) + " lives on another device than the plan");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr) == hipSuccess && base) {
        size_t used = (size_t)((const char *)ptr - (const char *)base);
        if (used > size || size - used < bytes)
            return fail(SHT_EINVAL, std::string(name) + " is smaller than the transform needs");
    } else {
        (void)hipGetLastError();
    }
    if (((uintptr_t)ptr & 15) != 0) return fail(SHT_EINVAL, std::string(name) + " is not 16-byte aligned");
    return SHT_OK;
}
}  // namespace sht

namespace {

int check_plan(const sht_plan_t *p) {
    if (!p) return fail(SHT_EINVAL, "plan is NULL");
    if (p->device < 0) return fail(SHT_EDEVICE, "host-only plan cannot execute transforms");
    return SHT_OK;
}

size_t nalm_of(int L) { return (size_t)(L + 1) * (L + 2) / 2; }
size_t npix_of(int N) { return 12ull * N * N; }
size_t q_bytes(const sht_plan_t *p, int B) { return (size_t)(p->L + 1) * p->nrings * B * 16; }

bool use_bf(const sht_plan_t *p, int path) {
    return p->bf.built && (path == SHT_PATH_BUTTERFLY || path == SHT_PATH_AUTO);
}

bool use_ip(const sht_plan_t *p, int path) { return p->ip.built && path == SHT_PATH_INTERP; }

size_t synth_ws_bytes(const sht_plan_t *p, const sht_exec_opts *x) {
    return sht::synth_ws_bytes_impl(p, x->nmaps, x->path, x->precision);
}

int check_exec(const sht_plan_t *p, const sht_exec_opts *x) {
    if (!x) return fail(SHT_EINVAL, "exec opts is NULL");
    if (x->nmaps < 1) return fail(SHT_EINVAL, "nmaps must be >= 1");
    if (x->path != SHT_PATH_AUTO && x->path != SHT_PATH_BRUTE && x->path != SHT_PATH_BUTTERFLY &&
        x->path != SHT_PATH_INTERP)
        return fail(SHT_EINVAL, "unknown path");
    if (x->path == SHT_PATH_BUTTERFLY && !p->bf.built)
        return fail(SHT_EUNSUPPORTED, "the butterfly path needs a plan built with eps > 0");
    if (x->path == SHT_PATH_INTERP && !p->ip.built)
        return fail(SHT_EUNSUPPORTED, "the interpolation path needs a plan built with interp = 1");
    if (x->precision != SHT_PREC_FP64 && x->precision != SHT_PREC_FP32)
        return fail(SHT_EINVAL, "unknown precision");
    if (x->precision == SHT_PREC_FP32 && !p->d_bf_T32)
        return fail(SHT_EUNSUPPORTED, "FP32 butterfly products need a plan built with store_fp32 = 1");
    return SHT_OK;
}

// Stream-ordered scratch: the caller's workspace or a temporary allocation.
struct Scratch {
    void *ptr = nullptr;
    bool owned = false;
    hipStream_t st = nullptr;
    int get(const sht_exec_opts *x, size_t bytes, int dev) {
        st = (hipStream_t)x->stream;
        if (x->workspace) {
            if (x->workspace_bytes < bytes)
                return fail(SHT_ENOMEM, "workspace smaller than sht_workspace_bytes()");
            int rc = check_dev_ptr(x->workspace, bytes, dev, "workspace");
            if (rc) return rc;
            ptr = x->workspace;
            return SHT_OK;
        }
        hipError_t e = hipMallocAsync(&ptr, bytes, st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ptr = nullptr;
            return fail(SHT_ENOMEM, std::string("workspace allocation: ") + hipGetErrorString(e));
        }
        owned = true;
        return SHT_OK;
    }
    ~Scratch() {
        if (owned && ptr) (void)hipFreeAsync(ptr, st);
    }
};

// Record the caller's stage event (before: which = 0, after: which = 1).
void stage_event(const sht_exec_opts *x, int stage, int which) {
    if (!x->stage_events) return;
    void *ev = x->stage_events[2 * stage + which];
    if (ev) (void)hipEventRecord((hipEvent_t)ev, (hipStream_t)x->stream);
}

int hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return SHT_OK;
    return fail(SHT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

namespace sht {
size_t synth_ws_bytes_impl(const sht_plan_s *p, int nmaps, int path, int precision) {
    size_t b = q_bytes(p, nmaps);
    if (use_bf(p, path)) b += bf_scratch_bytes(p, nmaps, precision == SHT_PREC_FP32);
    if (use_ip(p, path)) b += interp_scratch_bytes(p, nmaps);
    return b;
}

// Legendre phase of one synthesis on stream st into q = ws (the first
// q_bytes of the synth_ws_bytes_impl() bytes of ws).
static int legendre_stage(const sht_plan_s *p, int B, int path, int precision, const double *alm, void *ws,
                          hipStream_t st, const sht_exec_opts *x) {
    int rc;
    double *q = (double *)ws;
    if (use_ip(p, path)) {
        void *scr = (char *)ws + q_bytes(p, B);
        if ((rc = hip_status(launch_interp(p, B, alm, q, scr, st), "interpolation kernel launch"))) return rc;
    } else if (use_bf(p, path)) {
        void *scr = (char *)ws + q_bytes(p, B);
        if ((rc = hip_status(launch_butterfly(p, B, alm, q, scr, precision == SHT_PREC_FP32, st,
                                              x ? x->stage_events : nullptr),
                             "butterfly kernel launch")))
            return rc;
    } else if ((rc = hip_status(launch_legendre(p, B, alm, q, st), "Legendre kernel launch"))) {
        return rc;
    }
    return SHT_OK;
}

// Legendre phase and ring stage of one synthesis on stream st; ws holds
// synth_ws_bytes_impl() bytes.  Events of x (if any) bracket the stages.
static int synth_stages(const sht_plan_s *p, int B, int path, int precision, const double *alm, double *map,
                        void *ws, hipStream_t st, const sht_exec_opts *x) {
    int rc;
    double *q = (double *)ws;
    if (x) stage_event(x, SHT_STAGE_LEGENDRE, 0);
    if ((rc = legendre_stage(p, B, path, precision, alm, ws, st, x))) return rc;
    if (x) stage_event(x, SHT_STAGE_LEGENDRE, 1);
    if (x) stage_event(x, SHT_STAGE_RING, 0);
    rc = hip_status(launch_ring_synthesis(p, B, q, map, st), "ring kernel launch");
    if (x) stage_event(x, SHT_STAGE_RING, 1);
    return rc;
}

int synth_launch(const sht_plan_s *p, int nmaps, int path, int precision, const double *alm, double *map,
                 void *ws, hipStream_t st) {
    return synth_stages(p, nmaps, path, precision, alm, map, ws, st, nullptr);
}

// Polarized synthesis workspace: the six coefficient sets per map, the
// scalar synthesis workspace of 6 nmaps maps (its Legendre phase first), and
// the Q/U Legendre phase of 2 nmaps maps.
size_t pol_ws_bytes_impl(const sht_plan_s *p, int nmaps, int path, int precision) {
    return pol_alm_bytes(p, nmaps) + synth_ws_bytes_impl(p, 6 * nmaps, path, precision) + q_bytes(p, 2 * nmaps);
}
}  // namespace sht

namespace {
}  // namespace

extern "C" {

void sht_plan_opts_default(sht_plan_opts *o) {
    if (!o) return;
    o->cutoff = 1e-30;
    o->dd_sin = -1.0;
    o->nthreads = 0;
    o->rings_per_lane = 0;
    o->ring_threads = 0;
    o->host_only = 0;
    o->rho = 0.0;
    o->max_levels = -1;
    o->chunk = 0;
    o->id_safety = 0.0;
    o->store_fp32 = 0;
    o->batch_mib = 0;
    o->store_transpose = 0;
    o->interp = 0;
}

void sht_exec_opts_default(sht_exec_opts *o) {
    if (!o) return;
    o->nmaps = 1;
    o->path = SHT_PATH_AUTO;
    o->stream = nullptr;
    o->workspace = nullptr;
    o->workspace_bytes = 0;
    o->adjoint_convention = SHT_ADJ_TRANSPOSE;
    o->precision = SHT_PREC_FP64;
    o->stage_events = nullptr;
}

const char *sht_last_error(void) { return sht::last_error(); }

int sht_last_status(void) { return sht::last_status(); }

int sht_sync_status(const sht_plan_t *p, void *stream) {
    int rc = check_plan(p);
    if (rc) return rc;
    DeviceGuard g(p->device);
    if (!g.ok) return fail(SHT_EDEVICE, "cannot select the plan's device");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipGetLastError();
    return hip_status(e, "device work on the stream");
}

sht_plan_t *sht_plan(int L, int nside, double eps) { return sht_plan_ex(L, nside, eps, nullptr); }

sht_plan_t *sht_plan_ex(int L, int nside, double eps, const sht_plan_opts *opts) {
    auto t0 = std::chrono::steady_clock::now();
    if (L < 0 || L > 16383) {
        fail(SHT_EINVAL, "L must be in [0, 16383]");
        return nullptr;
    }
    if (nside < 1 || nside > 2048) {
        fail(nside < 1 ? SHT_EINVAL : SHT_EUNSUPPORTED, "nside must be in [1, 2048]");
        return nullptr;
    }
    if (!(eps >= 0.0)) {
        fail(SHT_EINVAL, "eps must be >= 0");
        return nullptr;
    }
    if (eps >= 1e-2) {
        fail(SHT_EINVAL, "eps must be below 1e-2");
        return nullptr;
    }
    sht_plan_opts o;
    sht_plan_opts_default(&o);
    if (opts) o = *opts;
    if (o.max_levels < -1 || o.max_levels > kBfMaxLv || o.chunk < 0 || o.chunk > 4096) {
        fail(SHT_EINVAL, "max_levels must be in [-1, 10] and chunk in [0, 4096]");
        return nullptr;
    }
    if (!(o.cutoff > 0.0) || o.cutoff > 1e-10) {
        fail(SHT_EINVAL, "cutoff must be in (0, 1e-10]");
        return nullptr;
    }
    sht_plan_s *p = new (std::nothrow) sht_plan_s();
    if (!p) {
        fail(SHT_ENOMEM, "out of host memory");
        return nullptr;
    }
    p->L = L;
    p->nside = nside;
    p->eps = eps;
    p->opts = o;
    int rc;
    try {
        rc = build_host_tables(p);
    } catch (const std::bad_alloc &) {
        rc = fail(SHT_ENOMEM, "out of host memory while building the plan");
    }
    if (rc != SHT_OK) {
        delete p;
        return nullptr;
    }
    if (!o.host_only) {
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
            (void)hipGetLastError();
            fail(SHT_EDEVICE, "no HIP device available");
            delete p;
            return nullptr;
        }
        p->device = dev;
        if (upload_tables(p) != SHT_OK) {
            delete p;
            return nullptr;
        }
        void *scr = nullptr;  // look up the no-allocation scratch of this device now
        if (noalloc_scratch(dev, &scr) != SHT_OK) {
            sht_plan_free(p);
            return nullptr;
        }
    }
    p->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return p;
}

void sht_plan_free(sht_plan_t *p) {
    if (!p) return;
    if (p->device >= 0) {
        DeviceGuard g(p->device);
        free_device_tables(p);
    }
    delete p;
}

int sht_plan_info(const sht_plan_t *p, sht_plan_info_t *out) {
    if (!p || !out) return fail(SHT_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->L = p->L;
    out->nside = p->nside;
    out->nrings = p->nrings;
    out->n_dd_rings = p->n_dd_rings;
    out->eps = p->eps;
    out->n_step = p->n_step;
    out->n_step_exec = p->n_step_exec;
    out->n_step_dd = p->n_step_dd;
    out->n_step_lanes = p->n_step_lanes;
    out->device_bytes = p->device_bytes;
    out->build_seconds = p->build_seconds;
    const BflyPlan &b = p->bf;
    out->bf_built = b.built;
    if (b.built) {
        out->bf_T_entries = b.T_entries;
        out->bf_res_elems = b.res_elems;
        out->bf_nodes = b.n_nodes;
        out->bf_units = b.n_units;
        out->bf_res_lanes = b.n_res_lanes;
        out->bf_res_exec = b.res_exec;
        for (int i = 0; i <= kBfMaxLv; i++) out->bf_depth_hist[i] = b.depth_hist[i];
        out->bf_build_seconds = b.build_seconds;
        out->bf_nbatch = b.nbatch;
        for (int i = 0; i <= kBfMaxLv; i++) {
            out->bf_level_T[i] = b.level_T[i];
            out->bf_level_units[i] = b.level_units[i];
            out->bf_level_nodes[i] = b.level_nodes[i];
        }
    }
    out->ip_built = p->ip.built;
    out->ip_nodes = p->ip.nodes;
    out->ip_steps = p->ip.steps;
    out->ip_exec = p->ip.exec;
    out->ip_build_seconds = p->ip.build_seconds;
    out->ip_direct = p->ip.direct;
    out->pol_rings = p->pol_n;
    return SHT_OK;
}

size_t sht_workspace_bytes(const sht_plan_t *p, const sht_exec_opts *x) {
    if (!p || !x || x->nmaps < 1) return 0;
    return synth_ws_bytes(p, x);
}

int sht_synthesis(const sht_plan_t *p, const double *alm, double *map) {
    sht_exec_opts x;
    sht_exec_opts_default(&x);
    return sht_synthesis_ex(p, &x, alm, map);
}

int sht_synthesis_ex(const sht_plan_t *p, const sht_exec_opts *x, const double *alm, double *map) {
    int rc = check_plan(p);
    if (!rc) rc = check_exec(p, x);
    if (rc) return rc;
    DeviceGuard g(p->device);
    if (!g.ok) return fail(SHT_EDEVICE, "cannot select the plan's device");
    const int B = x->nmaps;
    if ((rc = check_dev_ptr(alm, nalm_of(p->L) * B * 16, p->device, "alm"))) return rc;
    if ((rc = check_dev_ptr(map, npix_of(p->nside) * B * 8, p->device, "map"))) return rc;
    Scratch ws;
    if ((rc = ws.get(x, synth_ws_bytes(p, x), p->device))) return rc;
    return synth_stages(p, B, x->path, x->precision, alm, map, ws.ptr, (hipStream_t)x->stream, x);
}

size_t sht_pol_workspace_bytes(const sht_plan_t *p, const sht_exec_opts *x) {
    if (check_plan(p) || check_exec(p, x) || x->precision != SHT_PREC_FP64) return 0;
    return pol_ws_bytes_impl(p, x->nmaps, x->path, x->precision);
}

int sht_pol_synthesis(const sht_plan_t *p, const sht_exec_opts *x, const double *E, const double *B, double *QU) {
    int rc = check_plan(p);
    if (!rc) rc = check_exec(p, x);
    if (rc) return rc;
    if (p->L < 1) return fail(SHT_EINVAL, "polarized synthesis needs a plan with L >= 1 (band limit L - 1)");
    if (x->precision != SHT_PREC_FP64)
        return fail(SHT_EUNSUPPORTED, "polarized synthesis runs in FP64 (its combination divides by sin^2(theta))");
    DeviceGuard g(p->device);
    if (!g.ok) return fail(SHT_EDEVICE, "cannot select the plan's device");
    const int n = x->nmaps;
    if ((rc = check_dev_ptr(E, nalm_of(p->L - 1) * n * 16, p->device, "E"))) return rc;
    if ((rc = check_dev_ptr(B, nalm_of(p->L - 1) * n * 16, p->device, "B"))) return rc;
    if ((rc = check_dev_ptr(QU, npix_of(p->nside) * 2 * n * 8, p->device, "QU"))) return rc;
    Scratch ws;
    if ((rc = ws.get(x, pol_ws_bytes_impl(p, n, x->path, x->precision), p->device))) return rc;
    hipStream_t st = (hipStream_t)x->stream;
    char *base = (char *)ws.ptr;
    double *alm6 = (double *)base;
    void *sws = base + pol_alm_bytes(p, n);
    double *q6 = (double *)sws;
    double *q2 = (double *)((char *)sws + synth_ws_bytes_impl(p, 6 * n, x->path, x->precision));
    stage_event(x, SHT_STAGE_LEGENDRE, 0);
    if ((rc = hip_status(launch_pol_prep(p, n, E, B, alm6, st), "polarization coefficient launch"))) return rc;
    if ((rc = legendre_stage(p, 6 * n, x->path, x->precision, alm6, sws, st, nullptr))) return rc;
    if ((rc = hip_status(launch_pol_combine(p, n, q6, q2, st), "spin-2 combination launch"))) return rc;
    if ((rc = hip_status(launch_pol_polar(p, n, E, B, q2, st), "polar spin-2 launch"))) return rc;
    stage_event(x, SHT_STAGE_LEGENDRE, 1);
    stage_event(x, SHT_STAGE_RING, 0);
    rc = hip_status(launch_ring_synthesis(p, 2 * n, q2, QU, st), "ring kernel launch");
    stage_event(x, SHT_STAGE_RING, 1);
    return rc;
}

size_t sht_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int sht_synthesis_noalloc(const sht_plan_t *p, const sht_exec_opts *x, const double *alm, double *map) {
    int rc = check_plan(p);
    if (!rc) rc = check_exec(p, x);
    if (rc) return rc;
    DeviceGuard g(p->device);
    if (!g.ok) return fail(SHT_EDEVICE, "cannot select the plan's device");
    const int B = x->nmaps;
    const size_t need = synth_ws_bytes(p, x);
    if (need > kNoAllocScratchBytes)
        return fail(SHT_ENOMEM, "transform needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                    std::to_string(kNoAllocScratchBytes) + " of sht_synthesis_noalloc");
    if ((rc = check_dev_ptr(alm, nalm_of(p->L) * B * 16, p->device, "alm"))) return rc;
    if ((rc = check_dev_ptr(map, npix_of(p->nside) * B * 8, p->device, "map"))) return rc;
    void *scr = nullptr;
    if ((rc = noalloc_scratch(p->device, &scr))) return rc;
    return synth_stages(p, B, x->path, x->precision, alm, map, scr, (hipStream_t)x->stream, x);
}

int sht_adjoint(const sht_plan_t *p, const double *map, double *alm) {
    sht_exec_opts x;
    sht_exec_opts_default(&x);
    return sht_adjoint_ex(p, &x, map, alm);
}

static int check_conv(const sht_exec_opts *x) {
    if (x->adjoint_convention != SHT_ADJ_TRANSPOSE && x->adjoint_convention != SHT_ADJ_DAGGER)
        return fail(SHT_EINVAL, "unknown adjoint convention");
    return SHT_OK;
}

// Ring analysis and transposed Legendre phase of one adjoint on x->stream;
// ws holds synth_ws_bytes() bytes.
static int adjoint_stages(const sht_plan_t *p, const sht_exec_opts *x, double wpos, const double *map,
                          double *alm, void *ws) {
    int rc;
    const int B = x->nmaps;
    hipStream_t st = (hipStream_t)x->stream;
    double *ybar = (double *)ws;
    stage_event(x, SHT_STAGE_RING_ADJ, 0);
    if ((rc = hip_status(launch_ring_analysis(p, B, map, ybar, wpos, st), "ring analysis launch"))) return rc;
    stage_event(x, SHT_STAGE_RING_ADJ, 1);
    stage_event(x, SHT_STAGE_LEGENDRE_ADJ, 0);
    if (use_bf(p, x->path))
        rc = hip_status(launch_butterfly_adjoint(p, B, ybar, alm, (char *)ws + q_bytes(p, B),
                                                 x->precision == SHT_PREC_FP32, st),
                        "adjoint butterfly launch");
    else
        rc = hip_status(launch_legendre_adjoint(p, B, ybar, alm, st), "adjoint Legendre launch");
    stage_event(x, SHT_STAGE_LEGENDRE_ADJ, 1);
    return rc;
}

int sht_adjoint_ex(const sht_plan_t *p, const sht_exec_opts *x, const double *map, double *alm) {
    int rc = check_plan(p);
    if (!rc) rc = check_exec(p, x);
    if (!rc) rc = check_conv(x);
    if (!rc && x->path == SHT_PATH_INTERP) rc = fail(SHT_EUNSUPPORTED, "the interpolation path is synthesis only");
    if (rc) return rc;
    DeviceGuard g(p->device);
    if (!g.ok) return fail(SHT_EDEVICE, "cannot select the plan's device");
    const int B = x->nmaps;
    if ((rc = check_dev_ptr(map, npix_of(p->nside) * B * 8, p->device, "map"))) return rc;
    if ((rc = check_dev_ptr(alm, nalm_of(p->L) * B * 16, p->device, "alm"))) return rc;
    Scratch ws;
    if ((rc = ws.get(x, synth_ws_bytes(p, x), p->device))) return rc;
    const double wpos = x->adjoint_convention == SHT_ADJ_DAGGER ? 1.0 : 2.0;
    return adjoint_stages(p, x, wpos, map, alm, ws.ptr);
}

size_t sht_analysis_workspace_bytes(const sht_plan_t *p, const sht_exec_opts *x) {
    if (!p || !x || x->nmaps < 1) return 0;
    const size_t B = (size_t)x->nmaps;
    return synth_ws_bytes(p, x) + npix_of(p->nside) * B * 8 + nalm_of(p->L) * B * 16;
}

int sht_analysis_ex(const sht_plan_t *p, const sht_exec_opts *x, const double *map, double *alm, int iterations) {
    int rc = check_plan(p);
    if (!rc) rc = check_exec(p, x);
    if (!rc && x->path == SHT_PATH_INTERP) rc = fail(SHT_EUNSUPPORTED, "the interpolation path is synthesis only");
    if (rc) return rc;
    if (iterations < 0 || iterations > 1000) return fail(SHT_EINVAL, "iterations must be in [0, 1000]");
    DeviceGuard g(p->device);
    if (!g.ok) return fail(SHT_EDEVICE, "cannot select the plan's device");
    const int B = x->nmaps;
    const long long nmap = (long long)npix_of(p->nside) * B, nalm2 = (long long)nalm_of(p->L) * B * 2;
    if ((rc = check_dev_ptr(map, (size_t)nmap * 8, p->device, "map"))) return rc;
    if ((rc = check_dev_ptr(alm, (size_t)nalm2 * 8, p->device, "alm"))) return rc;
    Scratch ws;
    if ((rc = ws.get(x, sht_analysis_workspace_bytes(p, x), p->device))) return rc;
    hipStream_t st = (hipStream_t)x->stream;
    const size_t base = synth_ws_bytes(p, x);
    double *resid = (double *)((char *)ws.ptr + base);
    double *gin = (double *)((char *)ws.ptr + base + (size_t)nmap * 8);
    const double w = 4.0 * 3.14159265358979323846 / (double)npix_of(p->nside);
    // a = w Y^dagger f
    if ((rc = adjoint_stages(p, x, 1.0, map, alm, ws.ptr))) return rc;
    if ((rc = hip_status(launch_axpby(alm, alm, w, 0.0, nalm2, st), "analysis scale launch"))) return rc;
    for (int it = 0; it < iterations; it++) {
        // r = f - Y a;  a += w Y^dagger r
        if ((rc = synth_stages(p, B, x->path, x->precision, alm, resid, ws.ptr, st, nullptr))) return rc;
        if ((rc = hip_status(launch_axpby(resid, map, 1.0, -1.0, nmap, st), "analysis residual launch"))) return rc;
        if ((rc = adjoint_stages(p, x, 1.0, resid, gin, ws.ptr))) return rc;
        if ((rc = hip_status(launch_axpby(alm, gin, w, 1.0, nalm2, st), "analysis update launch"))) return rc;
    }
    return SHT_OK;
}

int sht_debug_ring_analysis(const sht_plan_t *p, const sht_exec_opts *x, const double *map, double *ybar) {
    int rc = check_plan(p);
    if (!rc) rc = check_exec(p, x);
    if (!rc) rc = check_conv(x);
    if (rc) return rc;
    DeviceGuard g(p->device);
    const int B = x->nmaps;
    if ((rc = check_dev_ptr(map, npix_of(p->nside) * B * 8, p->device, "map"))) return rc;
    if ((rc = check_dev_ptr(ybar, q_bytes(p, B), p->device, "ybar"))) return rc;
    const double wpos = x->adjoint_convention == SHT_ADJ_DAGGER ? 1.0 : 2.0;
    return hip_status(launch_ring_analysis(p, B, map, ybar, wpos, (hipStream_t)x->stream),
                      "ring analysis launch");
}

int sht_debug_legendre_adjoint(const sht_plan_t *p, const sht_exec_opts *x, const double *ybar, double *alm) {
    int rc = check_plan(p);
    if (!rc) rc = check_exec(p, x);
    if (rc) return rc;
    DeviceGuard g(p->device);
    const int B = x->nmaps;
    if ((rc = check_dev_ptr(ybar, q_bytes(p, B), p->device, "ybar"))) return rc;
    if ((rc = check_dev_ptr(alm, nalm_of(p->L) * B * 16, p->device, "alm"))) return rc;
    return hip_status(launch_legendre_adjoint(p, B, ybar, alm, (hipStream_t)x->stream),
                      "adjoint Legendre launch");
}

int sht_debug_interp_decomp(const double *A, int r, int c, double tol, int *k, int *piv, double *T) {
    if (!A || !k || !piv || !T || r < 1 || c < 1 || !(tol > 0)) return fail(SHT_EINVAL, "bad argument");
    std::vector<double> w(A, A + (size_t)r * c), Tv;
    std::vector<int> pv;
    *k = interp_decomp(w.data(), r, c, tol, 0.0, pv, Tv);
    std::memcpy(piv, pv.data(), sizeof(int) * c);
    std::memcpy(T, Tv.data(), sizeof(double) * Tv.size());
    return SHT_OK;
}

int sht_debug_butterfly_apply(const sht_plan_t *p, int m, int t, const double *x, double *y) {
    if (!p || !x || !y || m < 0 || m > p->L || t < 0 || t > 1) return fail(SHT_EINVAL, "bad argument");
    if (!p->bf.built) return fail(SHT_EUNSUPPORTED, "plan has no butterfly (eps = 0)");
    if (!p->bf.host_T_kept) return fail(SHT_EUNSUPPORTED, "interpolation data is on the device only");
    return butterfly_apply_host(p, m, t, x, y);
}

int sht_debug_interp_apply(const sht_plan_t *p, int m, int t, const double *x, double *y) {
    if (!p || !x || !y || m < 0 || m > p->L || t < 0 || t > 1) return fail(SHT_EINVAL, "bad argument");
    if (!p->ip.built) return fail(SHT_EUNSUPPORTED, "plan has no interpolation form (interp = 0)");
    return interp_apply_host(p, m, t, x, y);
}

int sht_debug_pol_column(const sht_plan_t *p, int m, int s, int k, double *out) {
    if (!p || !out) return fail(SHT_EINVAL, "bad argument");
    if (pol_column_host(p, m, s, k, out) != SHT_OK)
        return fail(SHT_EINVAL, "m must be in [0, L-1], s = +-2 and k a polar ring below sht_plan_info().pol_rings");
    return SHT_OK;
}

int sht_debug_butterfly_depth(const sht_plan_t *p, int m, int t) {
    if (!p || !p->bf.built || m < 0 || m > p->L || t < 0 || t > 1) return -1;
    return p->bf.depth[(size_t)2 * m + t];
}

int sht_debug_legendre_phase(const sht_plan_t *p, const sht_exec_opts *x, const double *alm, double *q) {
    int rc = check_plan(p);
    if (!rc) rc = check_exec(p, x);
    if (rc) return rc;
    DeviceGuard g(p->device);
    const int B = x->nmaps;
    if ((rc = check_dev_ptr(alm, nalm_of(p->L) * B * 16, p->device, "alm"))) return rc;
    if ((rc = check_dev_ptr(q, q_bytes(p, B), p->device, "q"))) return rc;
    return hip_status(launch_legendre(p, B, alm, q, (hipStream_t)x->stream), "Legendre kernel launch");
}

int sht_debug_ring_synthesis(const sht_plan_t *p, const sht_exec_opts *x, const double *q, double *map) {
    int rc = check_plan(p);
    if (!rc) rc = check_exec(p, x);
    if (rc) return rc;
    DeviceGuard g(p->device);
    const int B = x->nmaps;
    if ((rc = check_dev_ptr(q, q_bytes(p, B), p->device, "q"))) return rc;
    if ((rc = check_dev_ptr(map, npix_of(p->nside) * B * 8, p->device, "map"))) return rc;
    return hip_status(launch_ring_synthesis(p, B, q, map, (hipStream_t)x->stream), "ring kernel launch");
}

int sht_debug_coef(const sht_plan_t *p, int m, double *out) {
    if (!p || !out) return fail(SHT_EINVAL, "NULL argument");
    if (m < 0 || m > p->L) return fail(SHT_EINVAL, "m out of range");
    long long base = p->coef_off[m];
    for (int e = 0; e <= p->L - m; e++)
        for (int j = 0; j < 3; j++) out[3 * e + j] = p->coef_hi[4 * (base + e) + j];
    return SHT_OK;
}

int sht_debug_start(const sht_plan_t *p, int m, int t, int k, int *idx, double *vals) {
    if (!p || !idx || !vals) return fail(SHT_EINVAL, "NULL argument");
    if (m < 0 || m > p->L || t < 0 || t > 1 || k < 0 || k >= p->n_north)
        return fail(SHT_EINVAL, "index out of range");
    size_t row = (size_t)(2 * m + t);
    *idx = p->start_idx[row * p->n_north_pad + k];
    vals[0] = p->start_val[(row * 2 + 0) * p->n_north_pad + k];
    vals[1] = p->start_val[(row * 2 + 1) * p->n_north_pad + k];
    return SHT_OK;
}

}  // extern "C"
