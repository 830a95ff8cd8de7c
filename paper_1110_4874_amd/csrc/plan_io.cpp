// Plan files: the precomputed data written once and loaded by the library
// (Sec. 4.1 of the Wavemoth paper keeps its precomputed data in files that
// the core loads; Sec. 4.2 excludes that load from every timing).
//
// A file is a fixed header followed by a payload.  The header holds the
// operator's identity (L, nside, eps and the options that shape the plan),
// the library's record-layout constants, the payload length and two
// checksums (one over the header, one over the payload).  The payload is
// every host table of the plan in a fixed order: scalars as raw bytes,
// vectors as a 64-bit element count followed by their elements.  The same
// visitor walks the plan when saving and when loading, so the two cannot
// drift apart.  Integrity failures (truncation, a flipped bit, a foreign
// file) return SHT_ECORRUPT; a file written by a library with another
// record layout returns SHT_EUNSUPPORTED.
//
// Checksum: the payload is cut into units (each vector or scalar, and
// vectors further into 16 MiB blocks); each unit is hashed with four
// independent multiply-rotate lanes over 64-bit words, finished with the
// splitmix64 mixer (Steele, Lea and Flood, 2014), and the unit hashes are
// chained in order through the same mixer.  Every step is a bijection of
// the state for fixed input, so any change confined to one unit changes
// the final value.  Units are hashed on all host cores.
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstring>
#include <memory>

#include "internal.h"

namespace sht {
int check_dev_ptr(const void *ptr, size_t bytes, int dev, const char *name);
}

namespace {

using namespace sht;

constexpr char kMagic[8] = {'W', 'M', 'H', 'I', 'P', 'P', 'L', 'N'};
constexpr uint32_t kFileVersion = 6;
constexpr size_t kHashBlock = (size_t)16 << 20;

struct FileHeader {
    char magic[8];
    uint32_t version, header_bytes;
    uint64_t payload_bytes, payload_hash;
    int32_t L, nside;
    double eps, cutoff, dd_sin, rho, id_safety;
    int32_t max_levels, chunk, store_fp32, store_transpose, batch_mib, rings_per_lane, ring_threads, interp;
    int32_t layout[8];  // kLanes, kChunk, kCoefPad, kBfMaxLv, kBfNodeInts, kBfTaskRings, kBfPieceRings, 0
    uint64_t header_hash;  // over every byte above
};
static_assert(sizeof(FileHeader) == 152, "plan file header layout");

inline uint64_t mix64(uint64_t x) {
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}
inline uint64_t rotl(uint64_t x, int r) { return (x << r) | (x >> (64 - r)); }

uint64_t hash_bytes(const unsigned char *p, size_t n, uint64_t seed) {
    const uint64_t P1 = 0x9e3779b97f4a7c15ULL, P2 = 0xc2b2ae3d27d4eb4fULL;
    uint64_t h[4] = {seed ^ P1, seed ^ P2, seed + P1, seed - P2};
    size_t i = 0;
    for (; i + 32 <= n; i += 32)
        for (int j = 0; j < 4; j++) {
            uint64_t w;
            std::memcpy(&w, p + i + 8 * j, 8);
            h[j] = rotl(h[j] ^ (w * P1), 31) * P2;
        }
    for (; i < n; i += 8) {
        uint64_t w = 0;
        std::memcpy(&w, p + i, std::min<size_t>(8, n - i));
        h[0] = rotl(h[0] ^ (w * P1), 31) * P2;
    }
    return mix64(h[0]) ^ rotl(mix64(h[1]), 16) ^ rotl(mix64(h[2]), 32) ^ rotl(mix64(h[3]), 48) ^ (uint64_t)n;
}

struct Unit {
    const unsigned char *p;
    size_t n;
};

struct HashCtx {
    std::vector<Unit> units;
    std::vector<uint64_t> out;
};

void hash_worker(long i, void *vctx) {
    HashCtx *c = (HashCtx *)vctx;
    c->out[i] = hash_bytes(c->units[i].p, c->units[i].n, (uint64_t)i);
}

// The payload as a list of contiguous pieces, in file order.  Scalars are
// copied into owned storage; vector data is referenced in place.
struct Payload {
    std::vector<Unit> pieces;
    std::vector<std::unique_ptr<unsigned char[]>> owned;
    size_t bytes = 0;
    void add(const void *p, size_t n) {
        pieces.push_back({(const unsigned char *)p, n});
        bytes += n;
    }
    void add_copy(const void *p, size_t n) {
        owned.emplace_back(new unsigned char[n]);
        std::memcpy(owned.back().get(), p, n);
        add(owned.back().get(), n);
    }
    uint64_t hash(int nthreads) const {
        HashCtx c;
        for (const Unit &u : pieces) {
            if (u.n == 0) c.units.push_back(u);
            for (size_t o = 0; o < u.n; o += kHashBlock) c.units.push_back({u.p + o, std::min(kHashBlock, u.n - o)});
        }
        c.out.assign(c.units.size(), 0);
        parallel_for((long)c.units.size(), nthreads, hash_worker, &c);
        uint64_t h = 0x243f6a8885a308d3ULL;
        for (uint64_t v : c.out) h = mix64((h ^ v) + 0x9e3779b97f4a7c15ULL);
        return h;
    }
};

// Saving: records every field of the plan into a Payload.
struct Saver {
    Payload pl;
    template <typename T>
    void scalar(T &v) {
        pl.add_copy(&v, sizeof(T));
    }
    template <typename T>
    void vec(std::vector<T> &v) {
        uint64_t n = v.size();
        pl.add_copy(&n, 8);
        pl.add(v.data(), v.size() * sizeof(T));
    }
    template <typename T, size_t N>
    void arr(T (&a)[N]) {
        pl.add_copy(a, sizeof(a));
    }
    bool ok() const { return true; }
};

// Loading: reads every field in the same order, bounds-checked against the
// payload length the header declares; the pieces it fills are hashed after.
struct Loader {
    FILE *f = nullptr;
    uint64_t left = 0;
    bool good = true;
    Payload pl;
    template <typename T>
    void scalar(T &v) {
        if (!good) return;
        if (left < sizeof(T) || std::fread(&v, sizeof(T), 1, f) != 1) {
            good = false;
            return;
        }
        left -= sizeof(T);
        pl.add_copy(&v, sizeof(T));
    }
    template <typename T>
    void vec(std::vector<T> &v) {
        uint64_t n = 0;
        scalar(n);
        if (!good) return;
        if (n > left / sizeof(T)) {
            good = false;
            return;
        }
        v.resize((size_t)n);
        const size_t nb = (size_t)n * sizeof(T);
        size_t done = 0;
        while (done < nb) {  // large reads in pieces (some C libraries cap one fread)
            const size_t step = std::min(nb - done, (size_t)1 << 30);
            if (std::fread((char *)v.data() + done, 1, step, f) != step) {
                good = false;
                return;
            }
            done += step;
        }
        left -= nb;
        pl.add(v.data(), nb);
    }
    template <typename T, size_t N>
    void arr(T (&a)[N]) {
        if (!good) return;
        if (left < sizeof(a) || std::fread(a, sizeof(a), 1, f) != 1) {
            good = false;
            return;
        }
        left -= sizeof(a);
        pl.add_copy(a, sizeof(a));
    }
    bool ok() const { return good; }
};

// Every host table of the plan, in file order.  `T` is the interpolation
// data; a device plan that dropped its host copy passes a device read-back.
template <typename A>
void visit(A &ar, sht_plan_s *p, std::vector<double> &T) {
    ar.scalar(p->nrings);
    ar.scalar(p->n_north);
    ar.scalar(p->n_north_pad);
    ar.scalar(p->n_dd_pad);
    ar.scalar(p->n_dd_rings);
    ar.scalar(p->n_dd_groups);
    ar.scalar(p->rings_per_lane);
    ar.scalar(p->ring_threads);
    ar.scalar(p->n_step);
    ar.scalar(p->n_step_exec);
    ar.scalar(p->n_step_dd);
    ar.scalar(p->n_step_lanes);
    ar.scalar(p->tw_log);
    ar.scalar(p->build_seconds);
    ar.vec(p->z2_hi);
    ar.vec(p->z2_lo);
    ar.vec(p->ring_J);
    ar.vec(p->ring_s);
    ar.vec(p->ring_off);
    ar.vec(p->coef_off);
    ar.vec(p->coef_hi);
    ar.vec(p->coef_lo);
    ar.vec(p->start_idx);
    ar.vec(p->start_val);
    ar.vec(p->start_lo);
    ar.vec(p->grp_lo);
    ar.vec(p->grp_hi);
    ar.vec(p->tw);
    ar.vec(p->ring_M);
    ar.vec(p->ring_bs_off);
    ar.vec(p->bs_table);
    ar.vec(p->chirp);
    ar.vec(p->ring_chirp_off);
    ar.scalar(p->pol_n);
    ar.vec(p->pol_ring);
    ar.vec(p->pol_K);
    uint64_t ncls = p->classes.size();
    ar.scalar(ncls);
    if (!ar.ok() || ncls > 64) return;
    p->classes.resize((size_t)ncls);
    for (auto &c : p->classes) {
        int wrap = c.wrap ? 1 : 0;
        ar.scalar(c.lds_entries);
        ar.scalar(wrap);
        c.wrap = wrap != 0;
        ar.vec(c.rings);
    }
    InterpPlan &ip = p->ip;
    ar.scalar(ip.built);
    if (!ar.ok()) return;
    if (ip.built) {
        ar.vec(ip.node_off);
        ar.vec(ip.x_hi);
        ar.vec(ip.x_lo);
        ar.vec(ip.gam);
        ar.vec(ip.lamN);
        ar.vec(ip.sub);
        ar.vec(ip.lane);
        ar.vec(ip.val);
        ar.vec(ip.dd_task);
        ar.vec(ip.dd_lane);
        ar.vec(ip.dd_val);
        ar.vec(ip.patch);
        ar.scalar(ip.direct);
        ar.scalar(ip.nodes);
        ar.scalar(ip.dd_nodes);
        ar.scalar(ip.steps);
        ar.scalar(ip.exec);
        ar.scalar(ip.build_seconds);
    }
    BflyPlan &b = p->bf;
    ar.scalar(b.built);
    if (!ar.ok() || !b.built) return;
    ar.scalar(b.K);
    ar.scalar(b.ws_entries);
    ar.scalar(b.max_n);
    ar.vec(b.depth);
    ar.scalar(b.n_tasks);
    ar.vec(b.res_task);
    ar.vec(b.res_lane);
    ar.vec(b.res_val);
    ar.vec(b.res_sub);
    ar.scalar(b.nbatch);
    ar.vec(b.batch_count);
    ar.vec(b.batch_task);
    ar.vec(b.batch_sub);
    ar.vec(b.lv_off);
    ar.vec(b.lv_max_n);
    ar.vec(b.perm);
    ar.vec(b.node_i);
    ar.vec(T);
    ar.scalar(b.T_entries);
    ar.scalar(b.res_elems);
    ar.scalar(b.n_nodes);
    ar.scalar(b.n_res_lanes);
    ar.scalar(b.n_units);
    ar.arr(b.level_T);
    ar.arr(b.level_units);
    ar.arr(b.level_nodes);
    ar.vec(b.f1_unit);
    ar.vec(b.l1_plain);
    ar.vec(b.fold_slot);
    ar.vec(b.f1_off);
    ar.vec(b.l1_off);
    ar.vec(b.fold_off);
    ar.scalar(b.res_exec);
    ar.arr(b.depth_hist);
    ar.scalar(b.build_seconds);
}

void layout_of(int32_t *lay) {
    const int32_t v[8] = {kLanes, kChunk, kCoefPad, kBfMaxLv, kBfNodeInts, kBfTaskRings, kBfPieceRings, 0};
    std::memcpy(lay, v, sizeof(v));
}

uint64_t header_hash(const FileHeader &h) {
    return hash_bytes((const unsigned char *)&h, offsetof(FileHeader, header_hash), 0x5a5a5a5a);
}

// Cross-field consistency that the checksum cannot vouch for (a file from a
// buggy writer with a valid checksum must still not drive the kernels out of
// bounds): table sizes against the geometry the header states.
bool consistent(const sht_plan_s *p) {
    const size_t L = (size_t)p->L, np = (size_t)p->n_north_pad;
    if (p->nrings != 4 * p->nside - 1 || p->n_north != 2 * p->nside) return false;
    if (np % kLanes || np < (size_t)p->n_north) return false;
    if (p->ring_J.size() != (size_t)p->nrings || p->ring_s.size() != (size_t)p->nrings ||
        p->ring_off.size() != (size_t)p->nrings || p->ring_M.size() != (size_t)p->nrings)
        return false;
    if (p->z2_hi.size() != np || p->coef_off.size() != L + 2) return false;
    if ((size_t)p->coef_off[L + 1] * 4 != p->coef_hi.size() || p->coef_lo.size() != p->coef_hi.size()) return false;
    if (p->start_idx.size() != (L + 1) * 2 * np || p->start_val.size() != (L + 1) * 4 * np) return false;
    if (p->grp_lo.size() != (L + 1) * (np / kLanes)) return false;
    if (p->tw.size() != 2 * ((size_t)1 << (p->tw_log - 1))) return false;
    for (const auto &c : p->classes)
        for (int r : c.rings)
            if (r < 0 || r >= p->nrings) return false;
    if (p->pol_n < 0 || p->pol_n > p->n_north || p->pol_ring.size() != (size_t)p->pol_n * 6 ||
        p->pol_K.size() != (L + 1) * 8)
        return false;
    const InterpPlan &ip = p->ip;
    if (ip.built) {
        if (ip.node_off.size() != (L + 1) * 2 + 1 || (long long)ip.x_hi.size() != ip.nodes) return false;
        if (ip.node_off.back() != ip.nodes || ip.gam.size() != ip.x_hi.size() || ip.x_lo.size() != ip.x_hi.size())
            return false;
        if (ip.lamN.size() != (L + 1) * 2 * np || ip.sub.size() % 8 || ip.lane.size() != ip.val.size()) return false;
        if (ip.dd_task.size() % 8 || ip.dd_lane.size() * 2 != ip.dd_val.size()) return false;
        if (ip.patch.size() % 4) return false;
        for (size_t i = 0; i < ip.patch.size(); i += 4) {
            const int m = ip.patch[i], k = ip.patch[i + 1];
            if (m < 0 || m > (int)L || k < 0 || k >= p->n_north) return false;
            for (int t = 0; t < 2; t++) {
                const long long s = ip.patch[i + 2 + t];
                if (s < -1 || s >= ip.nodes) return false;
            }
        }
    }
    const BflyPlan &b = p->bf;
    if (b.built) {
        if (b.K != p->n_north || b.depth.size() != (L + 1) * 2 || b.nbatch < 1) return false;
        if (b.node_i.size() % kBfNodeInts || b.res_task.size() % 8 || b.res_sub.size() % 8) return false;
        if (b.lv_off.size() != (size_t)b.nbatch * (kBfMaxLv + 1) + 1) return false;
        if (b.batch_sub.size() != (size_t)b.nbatch + 1 || b.batch_task.size() != (size_t)b.nbatch + 1) return false;
        if (b.res_lane.size() != b.res_val.size()) return false;
    }
    return true;
}

int load_file(const char *path, const sht_plan_opts *lo, sht_plan_s **out) {
    *out = nullptr;
    if (!path) return fail(SHT_EINVAL, "path is NULL");
    struct stat st;
    if (stat(path, &st) != 0) return fail(SHT_EIO, std::string("cannot open plan file: ") + std::strerror(errno));
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(SHT_EIO, std::string("cannot open plan file: ") + std::strerror(errno));
    std::unique_ptr<FILE, int (*)(FILE *)> guard(f, std::fclose);
    FileHeader h;
    if (std::fread(&h, sizeof(h), 1, f) != 1) return fail(SHT_ECORRUPT, "plan file shorter than its header");
    if (std::memcmp(h.magic, kMagic, 8) != 0) return fail(SHT_ECORRUPT, "not a plan file (bad magic)");
    if (header_hash(h) != h.header_hash) return fail(SHT_ECORRUPT, "plan file header checksum mismatch");
    if (h.version != kFileVersion || h.header_bytes != sizeof(FileHeader))
        return fail(SHT_EUNSUPPORTED, "plan file version not supported by this library");
    int32_t lay[8];
    layout_of(lay);
    if (std::memcmp(lay, h.layout, sizeof(lay)) != 0)
        return fail(SHT_EUNSUPPORTED, "plan file written with another record layout");
    if ((uint64_t)st.st_size != sizeof(FileHeader) + h.payload_bytes)
        return fail(SHT_ECORRUPT, "plan file size does not match its header (truncated or extended)");
    if (h.L < 0 || h.L > 16383 || h.nside < 1 || h.nside > 2048 || !(h.eps >= 0.0))
        return fail(SHT_ECORRUPT, "plan file header out of range");
    std::unique_ptr<sht_plan_s> p(new (std::nothrow) sht_plan_s());
    if (!p) return fail(SHT_ENOMEM, "out of host memory");
    p->L = h.L;
    p->nside = h.nside;
    p->eps = h.eps;
    sht_plan_opts_default(&p->opts);
    p->opts.cutoff = h.cutoff;
    p->opts.dd_sin = h.dd_sin;
    p->opts.rho = h.rho;
    p->opts.id_safety = h.id_safety;
    p->opts.max_levels = h.max_levels;
    p->opts.chunk = h.chunk;
    p->opts.store_fp32 = h.store_fp32;
    p->opts.store_transpose = h.store_transpose;
    p->opts.batch_mib = h.batch_mib;
    p->opts.rings_per_lane = h.rings_per_lane;
    p->opts.ring_threads = h.ring_threads;
    p->opts.interp = h.interp;
    if (lo) {
        p->opts.host_only = lo->host_only;
        p->opts.store_fp32 = lo->store_fp32;
        p->opts.store_transpose = lo->store_transpose;
        p->opts.nthreads = lo->nthreads;
    }
    Loader ld;
    ld.f = f;
    ld.left = h.payload_bytes;
    try {
        visit(ld, p.get(), p->bf.T);
    } catch (const std::bad_alloc &) {
        return fail(SHT_ENOMEM, "out of host memory while reading the plan file");
    }
    if (!ld.good || ld.left != 0) return fail(SHT_ECORRUPT, "plan file payload truncated or malformed");
    if (ld.pl.hash(p->opts.nthreads) != h.payload_hash) return fail(SHT_ECORRUPT, "plan file payload checksum mismatch");
    if (!consistent(p.get())) return fail(SHT_ECORRUPT, "plan file tables inconsistent with its geometry");
    p->bf.host_T_kept = true;
    if (!p->opts.host_only) {
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
            (void)hipGetLastError();
            return fail(SHT_EDEVICE, "no HIP device available");
        }
        p->device = dev;
        int rc = upload_tables(p.get());
        if (rc != SHT_OK) return rc;
        void *scr = nullptr;  // look up the no-allocation scratch of this device now
        if ((rc = noalloc_scratch(dev, &scr)) != SHT_OK) {
            free_device_tables(p.get());
            return rc;
        }
    }
    *out = p.release();
    return SHT_OK;
}

}  // namespace

extern "C" {

int sht_plan_save(const sht_plan_t *cp, const char *path) {
    if (!cp || !path) return fail(SHT_EINVAL, "NULL argument");
    sht_plan_s *p = const_cast<sht_plan_s *>(cp);  // the visitor only reads when saving
    std::vector<double> Tdev;
    std::vector<double> *T = &p->bf.T;
    if (p->bf.built && !p->bf.host_T_kept) {
        // the host copy of the interpolation data was dropped after upload:
        // read it back from the device
        try {
            Tdev.resize((size_t)p->bf.T_entries);
        } catch (const std::bad_alloc &) {
            return fail(SHT_ENOMEM, "out of host memory for the interpolation data");
        }
        int prev = -1;
        (void)hipGetDevice(&prev);
        if (prev != p->device) (void)hipSetDevice(p->device);
        hipError_t e = hipMemcpy(Tdev.data(), p->d_bf_T, Tdev.size() * sizeof(double), hipMemcpyDeviceToHost);
        if (prev >= 0 && prev != p->device) (void)hipSetDevice(prev);
        if (e != hipSuccess) return fail(SHT_EDEVICE, std::string("plan read-back: ") + hipGetErrorString(e));
        T = &Tdev;
    }
    Saver sv;
    visit(sv, p, *T);
    FileHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kMagic, 8);
    h.version = kFileVersion;
    h.header_bytes = sizeof(FileHeader);
    h.payload_bytes = sv.pl.bytes;
    h.payload_hash = sv.pl.hash(p->opts.nthreads);
    h.L = p->L;
    h.nside = p->nside;
    h.eps = p->eps;
    h.cutoff = p->opts.cutoff;
    h.dd_sin = p->opts.dd_sin;
    h.rho = p->opts.rho;
    h.id_safety = p->opts.id_safety;
    h.max_levels = p->opts.max_levels;
    h.chunk = p->opts.chunk;
    h.store_fp32 = p->opts.store_fp32;
    h.store_transpose = p->opts.store_transpose;
    h.batch_mib = p->opts.batch_mib;
    h.rings_per_lane = p->opts.rings_per_lane;
    h.ring_threads = p->opts.ring_threads;
    h.interp = p->opts.interp;
    layout_of(h.layout);
    h.header_hash = header_hash(h);
    // write a temporary file next to the target and rename it into place,
    // so a reader never sees a partial file under the final name
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(SHT_EIO, std::string("cannot create plan file: ") + std::strerror(errno));
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
    for (const Unit &u : sv.pl.pieces) {
        for (size_t o = 0; ok && o < u.n; o += (size_t)1 << 30) {
            const size_t step = std::min(u.n - o, (size_t)1 << 30);
            ok = std::fwrite(u.p + o, 1, step, f) == step;
        }
        if (!ok) break;
    }
    const int err = errno;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) {
        std::remove(tmp.c_str());
        return fail(SHT_EIO, std::string("cannot write plan file: ") + std::strerror(err));
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        const int e2 = errno;
        std::remove(tmp.c_str());
        return fail(SHT_EIO, std::string("cannot rename plan file into place: ") + std::strerror(e2));
    }
    return SHT_OK;
}

sht_plan_t *sht_plan_load(const char *path) { return sht_plan_load_ex(path, nullptr); }

sht_plan_t *sht_plan_load_ex(const char *path, const sht_plan_opts *opts) {
    sht_plan_s *p = nullptr;
    int rc;
    try {
        rc = load_file(path, opts, &p);
    } catch (const std::bad_alloc &) {
        rc = fail(SHT_ENOMEM, "out of host memory while loading the plan");
    }
    return rc == SHT_OK ? p : nullptr;
}

}  // extern "C"
