// Work-queue batches: many synthesis requests of uneven size prepared once
// and replayed with a fixed, small number of launches (the many-transform
// regime of Sec. 3.4, where the paper notes that more simultaneous
// transforms need more blocking than it built).
//
// sht_batch_create splits every request into the work items of the
// brute-force Legendre phase, one per (pass of up to 4 maps, order m, ring
// block), estimates each item's cost from the plan's chain starts (chain
// steps times rings, compensated ring blocks weighted by their extra
// arithmetic), deals the items of each (pass, order) to one of eight lists,
// one per XCD, longest first, cuts each list into chunks that shrink along
// it (guided self-scheduling), and uploads them with one argument block per
// pass.  sht_batch_run then enqueues
//   1. one persistent Legendre launch: its waves take chunks of items from
//      a device counter, their own XCD's list first, then the others' (so
//      small requests fill in behind the long chains of large ones, with no
//      per-request launch and one atomic per chunk), and
//   2. one ring-FFT launch per ring size class, each covering that class's
//      rings of every request,
// all on the caller's stream, with no allocation and no host
// synchronisation, so a run can be captured into a HIP graph and replayed.
#include <algorithm>
#include <cstring>
#include <new>

#include "internal.h"

namespace sht {
int check_dev_ptr(const void *ptr, size_t bytes, int dev, const char *name);
}

using namespace sht;

namespace {

constexpr double kDdCost = 4.0;  // compensated step relative to an FP64 step

struct RingGroup {
    int lds_entries = 0;
    bool wrap = false;
    size_t lds = 0;
    RingArgs *d_args = nullptr;
    int2 *d_items = nullptr;
    long long nitems = 0;
    std::vector<RingArgs> args;   // per (request, class of this size)
    std::vector<int2> items;
};

// Butterfly path: the passes of one map-group width, with their stage
// launches in order.
struct BfStage {
    int stage = 0;          // 0 residual, 1 level nodes, 2 fused level-1 units, 3 fold blocks
    size_t lds = 0;
    long long n = 0;
    int2 *d_items = nullptr;
    std::vector<int2> items;
};
struct BfGroup {
    int nb = 0;
    void *d_args = nullptr;
    std::vector<char> args;
    std::vector<BfStage> stages;
};

}  // namespace

struct sht_batch_s {
    int device = -1;
    int n = 0;
    int path = SHT_PATH_BRUTE, fp32 = 0;
    std::vector<BfGroup> bf;
    int rings_per_lane = 2, ring_threads = 512;
    std::vector<sht_request> reqs;
    LegArgs *d_passes = nullptr;
    int4 *d_items = nullptr;
    unsigned *d_chunk_off = nullptr;  // chunk boundaries (item indices)
    unsigned *d_list_off = nullptr;   // [shape][9] list boundaries (chunk indices), one list per XCD
    unsigned *d_counter = nullptr;    // [shape][8] counters, 64 bytes apart
    long long nitems = 0, npasses = 0, nchunks = 0;
    int grid[kQueueShapes] = {};  // waves of each persistent Legendre launch (0: none)
    // fork/join over internal streams: independent launches of a run (wave
    // shapes, map-group widths, ring classes) overlap
    hipStream_t st[kMaxStreams] = {};
    hipEvent_t ev_fork[2] = {}, ev_join[2][kMaxStreams] = {};
    std::vector<RingGroup> groups;
};

namespace {

void free_batch(sht_batch_s *b) {
    if (!b) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (b->device >= 0 && prev != b->device) (void)hipSetDevice(b->device);
    if (b->d_passes) (void)hipFree(b->d_passes);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_counter) (void)hipFree(b->d_counter);
    if (b->d_list_off) (void)hipFree(b->d_list_off);
    if (b->d_chunk_off) (void)hipFree(b->d_chunk_off);
    for (auto &g : b->groups) {
        if (g.d_args) (void)hipFree(g.d_args);
        if (g.d_items) (void)hipFree(g.d_items);
    }
    for (auto &g : b->bf) {
        if (g.d_args) (void)hipFree(g.d_args);
        for (auto &st : g.stages)
            if (st.d_items) (void)hipFree(st.d_items);
    }
    for (int ph = 0; ph < 2; ph++) {
        if (b->ev_fork[ph]) (void)hipEventDestroy(b->ev_fork[ph]);
        for (int s = 0; s < kMaxStreams; s++)
            if (b->ev_join[ph][s]) (void)hipEventDestroy(b->ev_join[ph][s]);
    }
    if (prev >= 0 && prev != b->device) (void)hipSetDevice(prev);
    delete b;
}

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src) {
    hipError_t e = hipMalloc((void **)dst, std::max<size_t>(src.size(), 1) * sizeof(T));
    if (e == hipSuccess && !src.empty())
        e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

size_t q_bytes_of(const sht_request &q) {
    const size_t qb = (size_t)(q.plan->L + 1) * q.plan->nrings * q.nmaps * 16;
    return (qb + 255) / 256 * 256;
}

// Maps per pass on the butterfly path: 8, then 4, 2, 1.
int bf_pass_nb(int left) { return left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1; }

size_t bf_ws_bytes_of(const sht_plan_s *p, int nb, int fp32) {
    const size_t w = (size_t)p->bf.ws_entries * 2 * nb * (fp32 ? sizeof(float) : sizeof(double));
    return (w + 255) / 256 * 256;
}

// Workspace of a request: its Legendre phase, then on the butterfly path one
// vector workspace per pass (passes of a batch run concurrently).
size_t req_ws_bytes(const sht_request &q, int path, int fp32) {
    size_t b = q_bytes_of(q);
    if (path == SHT_PATH_BUTTERFLY)
        for (int m0 = 0; m0 < q.nmaps;) {
            const int nb = bf_pass_nb(q.nmaps - m0);
            b += bf_ws_bytes_of(q.plan, nb, fp32);
            m0 += nb;
        }
    return b;
}

int check_queue(const sht_request *reqs, int n, const sht_batch_opts *o, int *dev) {
    if (n < 1 || !reqs || !o) return fail(SHT_EINVAL, "a work-queue batch needs at least one request");
    if (o->path != SHT_PATH_BRUTE && o->path != SHT_PATH_BUTTERFLY)
        return fail(SHT_EUNSUPPORTED, "work-queue batches run the brute-force or the butterfly path");
    if (o->precision != SHT_PREC_FP64 && o->precision != SHT_PREC_FP32) return fail(SHT_EINVAL, "unknown precision");
    *dev = -1;
    for (int i = 0; i < n; i++) {
        const sht_plan_s *p = reqs[i].plan;
        if (!p || p->device < 0) return fail(SHT_EINVAL, "request without an executable plan");
        if (*dev < 0) *dev = p->device;
        if (p->device != *dev) return fail(SHT_EINVAL, "requests on different devices");
        if (reqs[i].nmaps < 1) return fail(SHT_EINVAL, "request with nmaps < 1");
        if (o->path == SHT_PATH_BUTTERFLY) {
            if (!p->bf.built) return fail(SHT_EUNSUPPORTED, "butterfly path asked for a plan built with eps = 0");
            if (p->bf.nbatch != 1)
                return fail(SHT_EUNSUPPORTED, "work-queue batches need plans whose orders run in one batch");
            if (o->precision == SHT_PREC_FP32 && !p->d_bf_T32)
                return fail(SHT_EUNSUPPORTED, "FP32 products asked for a plan without store_fp32");
        }
    }
    return SHT_OK;
}

struct Item {
    double cost;
    int4 w;      // {pass, m, ring block, first map}
    int shape;   // wave shape (queue_shape)
};

constexpr int kLists = 8;  // one work list per XCD

int build_bf(sht_batch_s *b, const sht_batch_opts *o) {
    const int fp32 = b->fp32;
    const size_t asz = bf_args_bytes(fp32);
    const int widths[4] = {8, 4, 2, 1};
    for (int wi = 0; wi < 4; wi++) {
        BfGroup g;
        g.nb = widths[wi];
        struct PassRef {
            const sht_plan_s *p;
        };
        std::vector<PassRef> refs;
        size_t off = 0;
        for (int r = 0; r < b->n; r++) {
            const sht_request &q = b->reqs[r];
            char *base = (char *)o->workspace + off;
            double *qbuf = reinterpret_cast<double *>(base);
            size_t woff = q_bytes_of(q);
            for (int m0 = 0; m0 < q.nmaps;) {
                const int nb = bf_pass_nb(q.nmaps - m0);
                if (nb == g.nb) {
                    g.args.resize(g.args.size() + asz);
                    bf_queue_args(q.plan, q.nmaps, m0, nb, fp32, q.alm, qbuf, base + woff, &g.args[g.args.size() - asz]);
                    refs.push_back({q.plan});
                }
                woff += bf_ws_bytes_of(q.plan, nb, fp32);
                m0 += nb;
            }
            off += req_ws_bytes(q, SHT_PATH_BUTTERFLY, fp32);
        }
        if (refs.empty()) continue;
        const int np = (int)refs.size();
        // residual pieces
        BfStage res;
        res.stage = 0;
        for (int i = 0; i < np; i++) {
            const BflyPlan &f = refs[i].p->bf;
            for (long long tk = f.batch_sub[0]; tk < f.batch_sub[1]; tk++) res.items.push_back(make_int2(i, (int)tk));
        }
        g.stages.push_back(std::move(res));
        // levels >= 2, deepest first
        for (int qv = 0; qv < kBfMaxLv - 1; qv++) {
            BfStage lv;
            lv.stage = 1;
            int wide = 0;
            for (int i = 0; i < np; i++) {
                const BflyPlan &f = refs[i].p->bf;
                for (long long nd = f.lv_off[qv]; nd < f.lv_off[qv + 1]; nd++) lv.items.push_back(make_int2(i, (int)nd));
                if (f.lv_off[qv + 1] > f.lv_off[qv]) wide = std::max(wide, f.lv_max_n[qv]);
            }
            lv.lds = bf_level_lds_bytes(wide, g.nb, fp32);
            if (!lv.items.empty()) g.stages.push_back(std::move(lv));
        }
        // level 1: nodes that run alone, then the fused units, then the fold
        BfStage l1, fu, fo;
        l1.stage = 1;
        fu.stage = 2;
        fo.stage = 3;
        int wide = 0;
        for (int i = 0; i < np; i++) {
            const BflyPlan &f = refs[i].p->bf;
            for (long long pp = f.l1_off[0]; pp < f.l1_off[1]; pp++) l1.items.push_back(make_int2(i, f.l1_plain[pp]));
            for (long long u = f.f1_off[0]; u < f.f1_off[1]; u++) fu.items.push_back(make_int2(i, (int)u));
            const long long nf = (f.fold_off[1] - f.fold_off[0]) * f.K * g.nb;
            for (long long blk = 0; blk < (nf + 255) / 256; blk++) fo.items.push_back(make_int2(i, (int)blk));
            wide = std::max(wide, f.lv_max_n[kBfMaxLv - 1]);
        }
        l1.lds = bf_level_lds_bytes(wide, g.nb, fp32);
        fu.lds = 2 * l1.lds;
        if (!l1.items.empty()) g.stages.push_back(std::move(l1));
        if (!fu.items.empty()) g.stages.push_back(std::move(fu));
        if (!fo.items.empty()) g.stages.push_back(std::move(fo));
        b->bf.push_back(std::move(g));
    }
    hipError_t e = hipSuccess;
    for (auto &g : b->bf) {
        if (e == hipSuccess) e = hipMalloc(&g.d_args, g.args.size());
        if (e == hipSuccess) e = hipMemcpy(g.d_args, g.args.data(), g.args.size(), hipMemcpyHostToDevice);
        for (auto &st : g.stages) {
            st.n = (long long)st.items.size();
            if (e == hipSuccess) e = upload(&st.d_items, st.items);
            std::vector<int2>().swap(st.items);
        }
    }
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EDEVICE,
                    std::string("batch tables: ") + hipGetErrorString(e));
    return SHT_OK;
}

int build_brute(sht_batch_s *b, const sht_batch_opts *o) {
    const int R = b->rings_per_lane;
    std::vector<LegArgs> passes;
    std::vector<Item> items;
    size_t off = 0;
    for (int r = 0; r < b->n; r++) {
        const sht_request &q = b->reqs[r];
        const sht_plan_s *p = q.plan;
        double *qbuf = reinterpret_cast<double *>((char *)o->workspace + off);
        off += req_ws_bytes(q, b->path, b->fp32);
        const int ng = p->n_north_pad / kLanes;
        for (int m0 = 0; m0 < q.nmaps;) {
            const int left = q.nmaps - m0, nb = left >= 4 ? 4 : left >= 2 ? 2 : 1;
            const LegArgs a = leg_args(p, q.nmaps, m0, R, q.alm, qbuf);
            const int pi = (int)passes.size();
            passes.push_back(a);
            const int nrb = a.dd_groups + a.fp_blocks;
            for (int m = 0; m <= p->L; m++) {
                const int n0 = (p->L - m) / 2 + 1;
                for (int rb = 0; rb < nrb; rb++) {
                    int lo = kDead, nrg;
                    double w;
                    const bool dd = rb < a.dd_groups;
                    if (dd) {
                        lo = p->grp_lo[(size_t)m * ng + rb];
                        nrg = 1;
                        w = kDdCost;
                    } else {
                        const int g0 = a.dd_groups + (rb - a.dd_groups) * R;
                        nrg = std::min(R, ng - g0);
                        for (int g = g0; g < g0 + nrg; g++) lo = std::min(lo, p->grp_lo[(size_t)m * ng + g]);
                        w = 1.0;
                    }
                    const double steps = lo < n0 ? (double)(n0 - lo) : 0.0;
                    // compensated waves take the maps two at a time
                    for (int b0 = 0; b0 < nb; b0 += dd ? 2 : nb) {
                        const int nw = dd ? std::min(2, nb - b0) : nb;
                        // chain steps (both parities) times rings, plus the stores
                        const double cost = w * steps * nrg * (5.0 + 4.0 * nw) + 64.0 * nrg * nw;
                        items.push_back({cost, make_int4(pi, m, rb, b0), queue_shape(dd, nw)});
                    }
                }
            }
            m0 += nb;
        }
    }
    if (items.size() > 0x7fffffffULL) return fail(SHT_EUNSUPPORTED, "batch has more than 2^31 work items");
    // per wave shape, the items of one (pass, m) go to one XCD's list:
    // groups dealt longest processing time first to the least loaded list,
    // then every list sorted longest item first and cut into chunks by
    // guided self-scheduling on the cost estimate (each chunk about 1/(2P)
    // of what is left of its list, P = waves whose home is the list, at
    // least one item)
    std::vector<int4> w;
    std::vector<unsigned> chunk_off, list_off((size_t)kQueueShapes * (kLists + 1), 0);
    hipError_t e = hipSuccess;
    for (int v = 0; v < kQueueShapes; v++) {
        std::vector<std::pair<double, long long>> groups;  // (cost, first item); a group's items are contiguous
        for (size_t i = 0; i < items.size();) {
            if (items[i].shape != v) {
                i++;
                continue;
            }
            size_t j = i;
            double c = 0.0;
            while (j < items.size() && items[j].w.x == items[i].w.x && items[j].w.y == items[i].w.y) {
                if (items[j].shape == v) c += items[j].cost;
                j++;
            }
            groups.push_back({c, (long long)i});
            i = j;
        }
        b->grid[v] = 0;
        if (groups.empty()) {
            for (int x = 0; x <= kLists; x++) list_off[(size_t)v * (kLists + 1) + x] = (unsigned)chunk_off.size();
            continue;
        }
        if (e == hipSuccess) e = legendre_queue_grid(v, R, &b->grid[v]);
        std::vector<size_t> order(groups.size());
        for (size_t i = 0; i < order.size(); i++) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t x, size_t y) { return groups[x].first > groups[y].first; });
        double load[kLists] = {};
        std::vector<std::vector<Item>> lists(kLists);
        for (size_t gi : order) {
            const int x = (int)(std::min_element(load, load + kLists) - load);
            load[x] += groups[gi].first;
            const long long i0 = groups[gi].second;
            for (long long i = i0;
                 i < (long long)items.size() && items[i].w.x == items[i0].w.x && items[i].w.y == items[i0].w.y; i++)
                if (items[i].shape == v) lists[x].push_back(items[i]);
        }
        const double P = std::max(b->grid[v] / kLists, 1);
        list_off[(size_t)v * (kLists + 1)] = (unsigned)chunk_off.size();
        for (int x = 0; x < kLists; x++) {
            std::stable_sort(lists[x].begin(), lists[x].end(),
                             [](const Item &a, const Item &b) { return a.cost > b.cost; });
            double left = 0.0;
            for (const Item &it : lists[x]) left += it.cost;
            double acc = 0.0, target = 0.0;
            for (size_t i = 0; i < lists[x].size(); i++) {
                if (acc == 0.0) {
                    chunk_off.push_back((unsigned)w.size());
                    target = left / (2.0 * P);
                }
                w.push_back(lists[x][i].w);
                acc += lists[x][i].cost;
                if (acc >= target) {
                    left -= acc;
                    acc = 0.0;
                }
            }
            list_off[(size_t)v * (kLists + 1) + x + 1] = (unsigned)chunk_off.size();
        }
    }
    std::vector<Item>().swap(items);
    if (e != hipSuccess) return fail(SHT_EDEVICE, std::string("queue grid: ") + hipGetErrorString(e));
    chunk_off.push_back((unsigned)w.size());
    b->nchunks = (long long)chunk_off.size() - 1;
    b->nitems = (long long)w.size();
    b->npasses = (long long)passes.size();
    e = upload(&b->d_passes, passes);
    if (e == hipSuccess) e = upload(&b->d_items, w);
    if (e == hipSuccess) e = upload(&b->d_chunk_off, chunk_off);
    if (e == hipSuccess) e = upload(&b->d_list_off, list_off);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_counter, (size_t)kQueueShapes * kLists * 64);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EDEVICE,
                    std::string("batch tables: ") + hipGetErrorString(e));
    return SHT_OK;
}

int build_rings(sht_batch_s *b, const sht_batch_opts *o) {
    // ring groups: one per (class size, wrap) over every request
    const int T = b->ring_threads;
    size_t off = 0;
    for (int r = 0; r < b->n; r++) {
        const sht_request &q = b->reqs[r];
        const sht_plan_s *p = q.plan;
        const double *qbuf = reinterpret_cast<const double *>((char *)o->workspace + off);
        off += req_ws_bytes(q, b->path, b->fp32);
        for (const auto &rc : p->classes) {
            RingGroup *g = nullptr;
            for (auto &x : b->groups)
                if (x.lds_entries == rc.lds_entries && x.wrap == rc.wrap) g = &x;
            if (!g) {
                b->groups.emplace_back();
                g = &b->groups.back();
                g->lds_entries = rc.lds_entries;
                g->wrap = rc.wrap;
            }
            RingArgs a = ring_args(p, q.nmaps, qbuf, q.map);
            a.rings = rc.d_rings;
            a.count = (int)rc.rings.size();
            g->lds = ring_class_shape(rc.lds_entries, rc.wrap, T, &a.fft_entries, &a.stage);
            const int ai = (int)g->args.size();
            g->args.push_back(a);
            for (int it = 0; it < a.count * q.nmaps; it++) g->items.push_back(make_int2(ai, it));
        }
    }
    hipError_t e = ring_queue_prepare(b->ring_threads);
    for (auto &g : b->groups) {
        g.nitems = (long long)g.items.size();
        if (g.nitems > 0x7fffffffLL && e == hipSuccess) e = hipErrorInvalidValue;
        if (e == hipSuccess) e = upload(&g.d_args, g.args);
        if (e == hipSuccess) e = upload(&g.d_items, g.items);
        std::vector<int2>().swap(g.items);
    }
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EDEVICE,
                    std::string("batch tables: ") + hipGetErrorString(e));
    return SHT_OK;
}

}  // namespace

extern "C" {

size_t sht_queue_workspace_bytes(const sht_request *reqs, int n, const sht_batch_opts *o) {
    int dev;
    if (check_queue(reqs, n, o, &dev) != SHT_OK) return 0;
    size_t off = 0;
    for (int i = 0; i < n; i++) off += req_ws_bytes(reqs[i], o->path, o->precision == SHT_PREC_FP32);
    return off;
}

sht_batch_t *sht_batch_create(const sht_request *reqs, int n, const sht_batch_opts *o) {
    int dev, rc;
    if ((rc = check_queue(reqs, n, o, &dev))) return nullptr;
    if (o->rings_per_lane != 0 && o->rings_per_lane != 1 && o->rings_per_lane != 2 && o->rings_per_lane != 4) {
        fail(SHT_EINVAL, "rings_per_lane must be 0, 1, 2 or 4");
        return nullptr;
    }
    if (o->ring_threads != 0 && o->ring_threads != 256 && o->ring_threads != 512 && o->ring_threads != 1024) {
        fail(SHT_EINVAL, "ring_threads must be 0, 256, 512 or 1024");
        return nullptr;
    }
    const size_t need = sht_queue_workspace_bytes(reqs, n, o);
    if (!o->workspace) {
        fail(SHT_EINVAL, "a work-queue batch needs a workspace of sht_queue_workspace_bytes()");
        return nullptr;
    }
    if (o->workspace_bytes < need) {
        fail(SHT_ENOMEM, "workspace smaller than sht_queue_workspace_bytes()");
        return nullptr;
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != dev && hipSetDevice(dev) != hipSuccess) {
        fail(SHT_EDEVICE, "cannot select the device");
        return nullptr;
    }
    struct Restore {
        int d;
        ~Restore() {
            if (d >= 0) (void)hipSetDevice(d);
        }
    } restore{prev != dev ? prev : -1};
    if (check_dev_ptr(o->workspace, need, dev, "workspace")) return nullptr;
    for (int i = 0; i < n; i++) {
        const sht_plan_s *p = reqs[i].plan;
        const int B = reqs[i].nmaps;
        if (check_dev_ptr(reqs[i].alm, (size_t)(p->L + 1) * (p->L + 2) / 2 * B * 16, dev, "alm")) return nullptr;
        if (check_dev_ptr(reqs[i].map, 12ull * p->nside * p->nside * B * 8, dev, "map")) return nullptr;
    }
    sht_batch_s *b = new (std::nothrow) sht_batch_s();
    if (!b) {
        fail(SHT_ENOMEM, "out of host memory");
        return nullptr;
    }
    b->device = dev;
    b->n = n;
    b->reqs.assign(reqs, reqs + n);
    b->rings_per_lane = o->rings_per_lane ? o->rings_per_lane : 2;
    b->ring_threads = o->ring_threads ? o->ring_threads : 512;
    b->path = o->path;
    b->fp32 = o->path == SHT_PATH_BUTTERFLY && o->precision == SHT_PREC_FP32;
    try {
        rc = b->path == SHT_PATH_BUTTERFLY ? build_bf(b, o) : build_brute(b, o);
        if (rc == SHT_OK) rc = build_rings(b, o);
        if (rc == SHT_OK) rc = pool_streams(dev, b->st);
        for (int ph = 0; ph < 2 && rc == SHT_OK; ph++) {
            bool ok = hipEventCreateWithFlags(&b->ev_fork[ph], hipEventDisableTiming) == hipSuccess;
            for (int s = 0; s < kMaxStreams && ok; s++)
                ok = hipEventCreateWithFlags(&b->ev_join[ph][s], hipEventDisableTiming) == hipSuccess;
            if (!ok) rc = fail(SHT_EDEVICE, "cannot create events");
        }
    } catch (const std::bad_alloc &) {
        rc = fail(SHT_ENOMEM, "out of host memory while building the batch");
    }
    if (rc != SHT_OK) {
        free_batch(b);
        return nullptr;
    }
    return b;
}

int sht_batch_run(const sht_batch_t *b, void *stream) {
    if (!b) return fail(SHT_EINVAL, "batch is NULL");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != b->device && hipSetDevice(b->device) != hipSuccess) return fail(SHT_EDEVICE, "cannot select the device");
    struct Restore {
        int d;
        ~Restore() {
            if (d >= 0) (void)hipSetDevice(d);
        }
    } restore{prev != b->device ? prev : -1};
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    // lanes of one phase fork from the caller's stream onto the internal
    // streams and join back into it (also after a failed launch, so that the
    // caller's stream stays consistent)
    auto fork = [&](int ph, int k) {
        if (hipEventRecord(b->ev_fork[ph], st) != hipSuccess) e = hipErrorLaunchFailure;
        for (int s = 0; s < k; s++) (void)hipStreamWaitEvent(b->st[s], b->ev_fork[ph], 0);
    };
    auto join = [&](int ph, int k) {
        for (int s = 0; s < k; s++) {
            (void)hipEventRecord(b->ev_join[ph][s], b->st[s]);
            (void)hipStreamWaitEvent(st, b->ev_join[ph][s], 0);
        }
    };
    // phase 0: the Legendre phase (brute force: one persistent launch per
    // wave shape; butterfly: the stages of each map-group width in order)
    if (b->path == SHT_PATH_BUTTERFLY) {
        const int k = std::min((int)b->bf.size(), kMaxStreams);
        fork(0, k);
        for (size_t gi = 0; gi < b->bf.size(); gi++) {
            const auto &g = b->bf[gi];
            for (const auto &sg : g.stages) {
                if (e != hipSuccess) break;
                e = launch_bf_queue_stage(sg.stage, g.nb, b->fp32, g.d_args, sg.d_items, sg.n, sg.lds,
                                          b->st[gi % kMaxStreams]);
            }
        }
        join(0, k);
    } else {
        e = launch_queue_reset(b->d_counter, st);
        fork(0, kQueueShapes);
        for (int v = 0; v < kQueueShapes && e == hipSuccess; v++)
            e = launch_legendre_queue(v, b->d_passes, b->d_items, b->d_chunk_off, b->d_list_off, b->d_counter,
                                      b->rings_per_lane, b->grid[v], b->st[v]);
        join(0, kQueueShapes);
    }
    // phase 1: one ring launch per ring size class
    const int kr = std::min((int)b->groups.size(), kMaxStreams);
    fork(1, kr);
    for (size_t gi = 0; gi < b->groups.size(); gi++) {
        if (e != hipSuccess) break;
        const auto &g = b->groups[gi];
        e = launch_ring_queue(b->ring_threads, g.d_args, g.d_items, g.nitems, g.lds, b->st[gi % kMaxStreams]);
    }
    join(1, kr);
    if (e != hipSuccess) return fail(SHT_EDEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    return SHT_OK;
}

int sht_batch_stats(const sht_batch_t *b, long long *items, int *launches, int *waves) {
    if (!b || !items || !launches || !waves) return fail(SHT_EINVAL, "NULL argument");
    *items = b->nitems;
    // counter reset, one Legendre launch per wave shape present, one per ring class
    *launches = 1 + (int)b->groups.size();
    *waves = 0;
    for (int v = 0; v < kQueueShapes; v++) {
        *launches += b->grid[v] > 0;
        *waves += b->grid[v];
    }
    if (b->path == SHT_PATH_BUTTERFLY) {
        *items = 0;
        *launches = (int)b->groups.size();
        for (const auto &g : b->bf)
            for (const auto &sg : g.stages) {
                *items += sg.n;
                (*launches)++;
            }
    }
    return SHT_OK;
}

void sht_batch_free(sht_batch_t *b) { free_batch(b); }

}  // extern "C"
