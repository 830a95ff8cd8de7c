// Batched synthesis of many independent requests (the many-transform
// regime of Sec. 3.4): requests are ordered by estimated work, longest
// first, and dealt to the least-loaded of a few internal streams that fork
// from and join back into the caller's stream through events, so that small
// transforms run concurrently with large ones.  Every launch is stream
// ordered and the call allocates nothing when given a workspace, so a whole
// batch can be captured into one HIP graph on the caller's stream.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace sht {
int check_dev_ptr(const void *ptr, size_t bytes, int dev, const char *name);
size_t synth_ws_bytes_impl(const sht_plan_s *p, int nmaps, int path, int precision);
int synth_launch(const sht_plan_s *p, int nmaps, int path, int precision, const double *alm, double *map,
                 void *ws, hipStream_t st);
}  // namespace sht

using namespace sht;

namespace {

struct Pool {
    int device = -1;
    hipStream_t s[kMaxStreams] = {};
};
std::mutex g_pool_mu;
std::vector<Pool> g_pools;

}  // namespace

// Default-priority, non-blocking internal streams of device dev (created on
// first use, with dev current, and kept until the process ends).
int sht::pool_streams(int dev, hipStream_t *out) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto &pl : g_pools)
        if (pl.device == dev) {
            std::memcpy(out, pl.s, sizeof(pl.s));
            return SHT_OK;
        }
    Pool pl;
    pl.device = dev;
    for (int i = 0; i < kMaxStreams; i++)
        if (hipStreamCreateWithFlags(&pl.s[i], hipStreamNonBlocking) != hipSuccess)
            return fail(SHT_EDEVICE, "cannot create internal streams");
    g_pools.push_back(pl);
    std::memcpy(out, pl.s, sizeof(pl.s));
    return SHT_OK;
}

namespace {

double work_of(const sht_request &r) {
    const sht_plan_s *p = r.plan;
    const double B = r.nmaps;
    // FP64 flops of the Legendre phase plus the ring stage's bytes (at ~50 flops per byte)
    return (double)p->n_step * (5.0 + 4.0 * B) + 50.0 * (double)(p->L + 1) * p->nrings * 16.0 * B;
}

struct Assignment {
    int ns = 1;
    std::vector<int> order;     // request indices, longest first
    std::vector<int> stream;    // per request: internal stream
    std::vector<size_t> ws_off; // per stream: workspace offset
    size_t total = 0;
};

int assign(const sht_request *reqs, int n, const sht_batch_opts *o, Assignment *a) {
    a->ns = o->nstreams > 0 ? std::min(o->nstreams, kMaxStreams) : 4;
    a->order.resize(n);
    for (int i = 0; i < n; i++) a->order[i] = i;
    std::stable_sort(a->order.begin(), a->order.end(),
                     [&](int x, int y) { return work_of(reqs[x]) > work_of(reqs[y]); });
    std::vector<double> load(a->ns, 0.0);
    std::vector<size_t> wsmax(a->ns, 0);
    a->stream.assign(n, 0);
    for (int i : a->order) {
        int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        a->stream[i] = s;
        load[s] += work_of(reqs[i]);
        wsmax[s] = std::max(wsmax[s], synth_ws_bytes_impl(reqs[i].plan, reqs[i].nmaps, o->path, o->precision));
    }
    a->ws_off.assign(a->ns, 0);
    size_t off = 0;
    for (int s = 0; s < a->ns; s++) {
        a->ws_off[s] = off;
        off += (wsmax[s] + 255) / 256 * 256;
    }
    a->total = off;
    return SHT_OK;
}

int check_requests(const sht_request *reqs, int n, const sht_batch_opts *o, int *dev) {
    if (n < 0 || (n > 0 && !reqs) || !o) return fail(SHT_EINVAL, "bad batch arguments");
    if (o->path != SHT_PATH_AUTO && o->path != SHT_PATH_BRUTE && o->path != SHT_PATH_BUTTERFLY)
        return fail(SHT_EINVAL, "unknown path");
    if (o->precision != SHT_PREC_FP64 && o->precision != SHT_PREC_FP32) return fail(SHT_EINVAL, "unknown precision");
    *dev = -1;
    for (int i = 0; i < n; i++) {
        const sht_plan_s *p = reqs[i].plan;
        if (!p || p->device < 0) return fail(SHT_EINVAL, "request without an executable plan");
        if (*dev < 0) *dev = p->device;
        if (p->device != *dev) return fail(SHT_EINVAL, "requests on different devices");
        if (reqs[i].nmaps < 1) return fail(SHT_EINVAL, "request with nmaps < 1");
        if (o->path == SHT_PATH_BUTTERFLY && !p->bf.built)
            return fail(SHT_EUNSUPPORTED, "butterfly path asked for a plan built with eps = 0");
        if (o->precision == SHT_PREC_FP32 && p->bf.built && !p->d_bf_T32)
            return fail(SHT_EUNSUPPORTED, "FP32 products asked for a plan without store_fp32");
    }
    return SHT_OK;
}

}  // namespace

extern "C" {

size_t sht_batch_workspace_bytes(const sht_request *reqs, int n, const sht_batch_opts *o) {
    int dev;
    if (check_requests(reqs, n, o, &dev) != SHT_OK || n == 0) return 0;
    Assignment a;
    assign(reqs, n, o, &a);
    return a.total;
}

void sht_batch_opts_default(sht_batch_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->nstreams = 4;
    o->path = SHT_PATH_AUTO;
    o->precision = SHT_PREC_FP64;
}

int sht_batch_execute(const sht_request *reqs, int n, const sht_batch_opts *o) {
    int dev, rc;
    if ((rc = check_requests(reqs, n, o, &dev))) return rc;
    if (n == 0) return SHT_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != dev && hipSetDevice(dev) != hipSuccess) return fail(SHT_EDEVICE, "cannot select the device");
    struct Restore {
        int d;
        ~Restore() {
            if (d >= 0) (void)hipSetDevice(d);
        }
    } restore{prev != dev ? prev : -1};
    for (int i = 0; i < n; i++) {
        const sht_plan_s *p = reqs[i].plan;
        const int B = reqs[i].nmaps;
        if ((rc = check_dev_ptr(reqs[i].alm, (size_t)(p->L + 1) * (p->L + 2) / 2 * B * 16, dev, "alm"))) return rc;
        if ((rc = check_dev_ptr(reqs[i].map, 12ull * p->nside * p->nside * B * 8, dev, "map"))) return rc;
    }
    Assignment a;
    assign(reqs, n, o, &a);
    if (!o->workspace) return fail(SHT_EINVAL, "a batch needs a workspace of sht_batch_workspace_bytes()");
    if (o->workspace_bytes < a.total) return fail(SHT_ENOMEM, "workspace smaller than sht_batch_workspace_bytes()");
    if ((rc = check_dev_ptr(o->workspace, a.total, dev, "workspace"))) return rc;
    hipStream_t st[kMaxStreams];
    if ((rc = pool_streams(dev, st))) return rc;
    hipStream_t caller = (hipStream_t)o->stream;
    // fork
    hipEvent_t fork_ev, join_ev[kMaxStreams];
    if (hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming) != hipSuccess)
        return fail(SHT_EDEVICE, "cannot create events");
    (void)hipEventRecord(fork_ev, caller);
    for (int s = 0; s < a.ns; s++) (void)hipStreamWaitEvent(st[s], fork_ev, 0);
    rc = SHT_OK;
    for (int i : a.order) {
        const int s = a.stream[i];
        rc = synth_launch(reqs[i].plan, reqs[i].nmaps, o->path, o->precision, reqs[i].alm, reqs[i].map,
                          (char *)o->workspace + a.ws_off[s], st[s]);
        if (rc) break;
    }
    // join (also after a failed launch, so the caller's stream stays consistent)
    for (int s = 0; s < a.ns; s++) {
        if (hipEventCreateWithFlags(&join_ev[s], hipEventDisableTiming) != hipSuccess) {
            rc = fail(SHT_EDEVICE, "cannot create events");
            join_ev[s] = nullptr;
            continue;
        }
        (void)hipEventRecord(join_ev[s], st[s]);
        (void)hipStreamWaitEvent(caller, join_ev[s], 0);
    }
    (void)hipEventDestroy(fork_ev);
    for (int s = 0; s < a.ns; s++)
        if (join_ev[s]) (void)hipEventDestroy(join_ev[s]);
    return rc;
}

}  // extern "C"
