// Host-side plan construction: every table the kernels read, computed once
// per (L, nside) in long double and rounded to double (or split into a
// double-double hi/lo pair where the compensated kernel needs it).
//
// What is precomputed follows App. A.2 of the Wavemoth paper: the
// coefficients of the two-step Legendre recurrence, and for every column
// z (ring) and parity the first Legendre values above the 1e-30 cutoff
// ("we increase k_start correspondingly"), so the kernels never touch the
// underflowing region.  The ring geometry is HEALPix (Gorski et al. 2005).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

#include "internal.h"

namespace sht {

typedef long double ld;
static const ld kPi = 3.14159265358979323846264338327950288L;

static thread_local std::string g_err;
static thread_local int g_status = 0;
void set_error(const std::string &msg) { g_err = msg; }
int fail(int code, const std::string &msg) {
    g_err = msg;
    g_status = code;
    return code;
}
const char *last_error() { return g_err.c_str(); }
int last_status() { return g_status; }

void parallel_for(long n, int nthreads, void (*fn)(long, void *), void *ctx) {
    if (n <= 0) return;
    if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
    nthreads = (int)std::max(1L, std::min<long>(nthreads, n));
    std::atomic<long> next(0);
    auto worker = [&]() {
        for (;;) {
            long i = next.fetch_add(1);
            if (i >= n) break;
            fn(i, ctx);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nthreads; t++) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
}

// ---------------------------------------------------------------------
// HEALPix RING geometry of ring i = 1..4N-1: z and sin^2(theta) from exact
// integer ratios, pixel count J, half-pixel shift s (phi_j = pi(2j+s)/J),
// first pixel index.
// ---------------------------------------------------------------------
static void ring_geometry(int N, int i, ld *z, ld *sin2, int *J, int *s, long long *off) {
    int ii = (i > 2 * N) ? 4 * N - i : i;  // northern counterpart
    ld zz, w;
    if (ii < N) {
        ld a = (ld)ii * ii, b = 3.0L * N * N;
        zz = (b - a) / b;
        w = a * (2.0L * b - a) / (b * b);
        *J = 4 * ii;
        *s = 1;
    } else {
        zz = (4.0L * N - 2.0L * ii) / (3.0L * N);
        w = (2.0L * ii - N) * (7.0L * N - 2.0L * ii) / (9.0L * N * N);
        *J = 4 * N;
        *s = ((ii - N) & 1) ? 0 : 1;
    }
    *z = (i > 2 * N) ? -zz : zz;
    *sin2 = w;
    long long NN = N;
    if (i < N)
        *off = 2LL * i * (i - 1);
    else if (i <= 3 * N)
        *off = 2 * NN * (NN - 1) + (long long)(i - N) * 4 * NN;
    else {
        long long ip = 4 * NN - i;
        *off = 12 * NN * NN - 2 * ip * (ip + 1);
    }
}

// ---------------------------------------------------------------------
// Two-step recurrence of App. A.2, Eq. A2:
//   P_{l+2} = (z^2 - d_l)/c_l P_l - c_{l-2}/c_l P_{l-2}
//           = (z^2 + alpha_l) beta_l P_l + gamma_l P_{l-2}
// with the paper's closed forms for c_l^m and d_l^m.  c_{l-2} vanishes for
// l = m, m+1, so both parity chains start from their first two values.
// ---------------------------------------------------------------------
static ld c_coef(int l, int m) {
    ld num = (ld)(l - m + 1) * (ld)(l - m + 2) * (ld)(l + m + 1) * (ld)(l + m + 2);
    ld den = (ld)(2 * l + 1) * (ld)(2 * l + 3) * (ld)(2 * l + 3) * (ld)(2 * l + 5);
    if (num <= 0) return 0;
    return sqrtl(num / den);
}
static ld d_coef(int l, int m) {
    return ((ld)2 * l * (l + 1) - (ld)2 * m * m - 1) / ((ld)(2 * l - 1) * (ld)(2 * l + 3));
}

struct BuildCtx {
    sht_plan_s *p;
    std::vector<ld> coefl;         // [entries][3] long double beta, alpha*beta, gamma
    std::vector<ld> zl, sinl;      // [n_north]
    std::atomic<int> bad{0};
    std::vector<long long> steps;  // per ring: executed steps
    std::vector<long long> alive;  // per ring: steps at or above the cutoff
    std::vector<long long> lane_steps;  // per m: lane-steps executed by the kernel
    bool keep_ld = false;               // butterfly: keep long-double starts
    std::vector<ld> start_ld;           // [(L+1)*2][2][n_north_pad]
};

static void coef_worker(long m, void *vctx) {
    BuildCtx *c = (BuildCtx *)vctx;
    sht_plan_s *p = c->p;
    long long base = p->coef_off[m];
    long long cnt = p->coef_off[m + 1] - base;
    for (long long e = 0; e < cnt; e++) {
        int l = (int)(m + e);
        ld cl = c_coef(l, (int)m), dl = d_coef(l, (int)m), cm2 = c_coef(l - 2, (int)m);
        ld beta = 1.0L / cl, ab = -dl / cl, gam = -cm2 / cl;
        ld vals[3] = {beta, ab, gam};
        for (int q = 0; q < 3; q++) {
            c->coefl[3 * (base + e) + q] = vals[q];
            double hi = (double)vals[q];
            p->coef_hi[4 * (base + e) + q] = hi;
            p->coef_lo[4 * (base + e) + q] = (double)(vals[q] - (ld)hi);
        }
        p->coef_hi[4 * (base + e) + 3] = 0.0;
        p->coef_lo[4 * (base + e) + 3] = 0.0;
    }
}

// Start values of every (m, parity) chain on north ring k.  The sectoral
// value P~_m^m = (-1)^m sqrt((2m+1)/(4pi) prod_{j<=m} (2j-1)/(2j)) sin^m
// is carried as mantissa * 2^E while m increases; each chain then runs
// through the region where P~ is below the cutoff (P~ grows with l there)
// and records the values at the last chunk boundary before it crosses.
static void start_worker(long k, void *vctx) {
    BuildCtx *c = (BuildCtx *)vctx;
    sht_plan_s *p = c->p;
    const int L = p->L, np = p->n_north_pad;
    const ld z = c->zl[k], z2 = z * z, st = c->sinl[k];
    const ld cutoff = (ld)p->opts.cutoff;
    const bool dd = k < p->n_dd_pad;
    ld v = 1.0L;
    long E = 0;
    long long steps = 0, alive = 0;
    for (int m = 0; m <= L; m++) {
        if (m > 0) {
            int ex;
            v *= st * sqrtl((ld)(2 * m - 1) / (ld)(2 * m));
            v = frexpl(v, &ex);
            E += ex;
        }
        ld pmm = v * sqrtl((ld)(2 * m + 1) / (4.0L * kPi));
        if (m & 1) pmm = -pmm;
        const ld *cf = c->coefl.data() + 3 * p->coef_off[m];
        for (int t = 0; t < 2; t++) {
            size_t row = (size_t)(2 * m + t);
            int nt = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
            int found = -1;
            ld s0 = 0, s1 = 0;
            long sE = 0;
            if (nt > 0 && v != 0.0L) {
                ld P0 = (t == 0) ? pmm : z * sqrtl((ld)(2 * m + 3)) * pmm;
                ld P1 = (z2 * cf[3 * t] + cf[3 * t + 1]) * P0;  // gamma = 0 at chain start
                long PE = E;
                for (int i = 0; i < nt; i++) {
                    if (i % kChunk == 0) {
                        s0 = P0;
                        s1 = P1;
                        sE = PE;
                    }
                    if (PE > -16000 && fabsl(ldexpl(P0, (int)PE)) >= cutoff) {
                        found = i - i % kChunk;
                        alive += nt - i;
                        break;
                    }
                    int e = t + 2 * i + 2;  // coefficients at l = m + t + 2(i+1)
                    ld P2 = (z2 * cf[3 * e] + cf[3 * e + 1]) * P1 + cf[3 * e + 2] * P0;
                    P0 = P1;
                    P1 = P2;
                    if (fabsl(P1) > 0x1p512L) {
                        P0 = ldexpl(P0, -512);
                        P1 = ldexpl(P1, -512);
                        PE += 512;
                    }
                }
            }
            if (found >= 0) {
                ld a = ldexpl(s0, (int)sE), b = ldexpl(s1, (int)sE);
                double ah = (double)a, bh = (double)b;
                // one of the pair may sit on a root of P~; the pair as a whole must
                // be far from the double underflow range
                if (fmax(fabs(ah), fabs(bh)) < 1e-290) c->bad.store(1);
                if (c->keep_ld) {
                    c->start_ld[(row * 2 + 0) * np + k] = a;
                    c->start_ld[(row * 2 + 1) * np + k] = b;
                }
                p->start_idx[row * np + k] = found;
                p->start_val[(row * 2 + 0) * np + k] = ah;
                p->start_val[(row * 2 + 1) * np + k] = bh;
                if (dd) {
                    p->start_lo[(row * 2 + 0) * p->n_dd_pad + k] = (double)(a - (ld)ah);
                    p->start_lo[(row * 2 + 1) * p->n_dd_pad + k] = (double)(b - (ld)bh);
                }
                steps += nt - found;
            }
        }
    }
    c->steps[k] = steps;
    c->alive[k] = alive;
}

static void group_worker(long m, void *vctx) {
    BuildCtx *c = (BuildCtx *)vctx;
    sht_plan_s *p = c->p;
    const int np = p->n_north_pad, ng = np / kLanes;
    const int n0 = (p->L - (int)m) / 2 + 1;
    for (int g = 0; g < ng; g++) {
        int lo = kDead, hi = -1;
        for (int t = 0; t < 2; t++)
            for (int k = g * kLanes; k < (g + 1) * kLanes; k++) {
                int s = p->start_idx[(size_t)(2 * m + t) * np + k];
                if (s < kDead) {
                    lo = std::min(lo, s);
                    hi = std::max(hi, s);
                }
            }
        p->grp_lo[(size_t)m * ng + g] = lo;
        p->grp_hi[(size_t)m * ng + g] = hi;
    }
    // lane-steps the kernel executes for this m (every lane of a wave runs
    // both parities from the wave's first chunk to the end of the chain)
    long long lanes = 0;
    const int R = p->rings_per_lane, gdd = p->n_dd_groups;
    for (int g0 = 0; g0 < ng; g0 += (g0 < gdd ? 1 : R)) {
        const int w = g0 < gdd ? 1 : std::min(R, ng - g0);
        int lo = kDead;
        for (int r = 0; r < w; r++) lo = std::min(lo, p->grp_lo[(size_t)m * ng + g0 + r]);
        if (lo < n0) lanes += 2LL * kLanes * w * (n0 - lo);
    }
    c->lane_steps[m] = lanes;
}

// ---------------------------------------------------------------------
// Ring FFT tables.
// ---------------------------------------------------------------------
static int ilog2(long long x) {
    int r = 0;
    while ((1LL << r) < x) r++;
    return r;
}
static bool is_pow2(long long x) { return x > 0 && (x & (x - 1)) == 0; }

// In-place iterative radix-2 FFT in long double, sign -1 (forward).
static void host_fft_forward(std::vector<ld> &re, std::vector<ld> &im) {
    size_t n = re.size();
    for (size_t i = 1, j = 0; i < n; i++) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            std::swap(re[i], re[j]);
            std::swap(im[i], im[j]);
        }
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        for (size_t k = 0; k < len / 2; k++) {
            ld ang = -2.0L * kPi * (ld)k / (ld)len;
            ld wr = cosl(ang), wi = sinl(ang);
            for (size_t b = 0; b < n; b += len) {
                size_t i0 = b + k, i1 = i0 + len / 2;
                ld tr = re[i1] * wr - im[i1] * wi, ti = re[i1] * wi + im[i1] * wr;
                re[i1] = re[i0] - tr;
                im[i1] = im[i0] - ti;
                re[i0] += tr;
                im[i0] += ti;
            }
        }
    }
}

struct BsCtx {
    sht_plan_s *p;
    std::vector<int> ns;            // distinct Bluestein sizes n
    std::vector<long long> offs;    // spectrum table offset per entry
    std::vector<long long> coffs;   // chirp table offset per entry
};

// Spectrum of the Bluestein chirp for a length-n DFT padded to M: the
// convolution kernel v_j = exp(-i pi j^2 / n), |j| < n, wrapped mod M.
// Stored bit-reversed (the order a decimation-in-frequency FFT leaves its
// output in) and scaled by 1/M.
static void bs_worker(long idx, void *vctx) {
    BsCtx *c = (BsCtx *)vctx;
    int n = c->ns[idx];
    int M = 1 << ilog2(2LL * n - 1);
    std::vector<ld> re(M, 0.0L), im(M, 0.0L);
    for (int j = 0; j < n; j++) {
        long long r = ((long long)j * j) % (2LL * n);
        ld ang = -kPi * (ld)r / (ld)n;
        re[j] = cosl(ang);
        im[j] = sinl(ang);
        if (j > 0) {
            re[M - j] = re[j];
            im[M - j] = im[j];
        }
    }
    // the chirp itself, w_k = exp(+i pi k^2 / n), k < n (pre- and post-multiplier)
    double *cw = c->p->chirp.data() + 2 * c->coffs[idx];
    for (int j = 0; j < n; j++) {
        long long r = ((long long)j * j) % (2LL * n);
        ld ang = kPi * (ld)r / (ld)n;
        cw[2 * j] = (double)cosl(ang);
        cw[2 * j + 1] = (double)sinl(ang);
    }
    host_fft_forward(re, im);
    int lg = ilog2(M);
    double *out = c->p->bs_table.data() + 2 * c->offs[idx];
    for (int q = 0; q < M; q++) {
        unsigned rev = 0;
        for (int b = 0; b < lg; b++)
            if (q & (1 << b)) rev |= 1u << (lg - 1 - b);
        out[2 * q] = (double)(re[rev] / (ld)M);
        out[2 * q + 1] = (double)(im[rev] / (ld)M);
    }
}

int build_host_tables(sht_plan_s *p) {
    const int L = p->L, N = p->nside;
    const int nth = p->opts.nthreads;
    p->rings_per_lane = (p->opts.rings_per_lane == 1 || p->opts.rings_per_lane == 4) ? p->opts.rings_per_lane : 2;
    p->ring_threads = (p->opts.ring_threads == 256 || p->opts.ring_threads == 1024) ? p->opts.ring_threads : 512;
    p->nrings = 4 * N - 1;
    p->n_north = 2 * N;
    p->n_north_pad = (p->n_north + kLanes - 1) / kLanes * kLanes;
    const int np = p->n_north_pad;

    BuildCtx ctx;
    ctx.p = p;
    // ring geometry
    p->ring_J.resize(p->nrings);
    p->ring_s.resize(p->nrings);
    p->ring_off.resize(p->nrings);
    p->z2_hi.assign(np, 0.0);
    p->z2_lo.assign(np, 0.0);
    ctx.zl.assign(np, 0.0L);
    ctx.sinl.assign(np, 0.0L);
    for (int i = 1; i <= p->nrings; i++) {
        ld z, s2;
        int J, s;
        long long off;
        ring_geometry(N, i, &z, &s2, &J, &s, &off);
        p->ring_J[i - 1] = J;
        p->ring_s[i - 1] = s;
        p->ring_off[i - 1] = off;
        if (i <= p->n_north) {
            ld z2 = z * z;
            p->z2_hi[i - 1] = (double)z2;
            p->z2_lo[i - 1] = (double)(z2 - (ld)(double)z2);
            ctx.zl[i - 1] = z;
            ctx.sinl[i - 1] = sqrtl(s2);
        }
    }
    // compensated-arithmetic rings: those nearest the poles
    double dd_sin = p->opts.dd_sin < 0 ? 0.1 * (double)L / 4095.0 : p->opts.dd_sin;
    int ndd = 0;
    while (ndd < p->n_north && (double)ctx.sinl[ndd] < dd_sin) ndd++;
    p->n_dd_rings = ndd;
    p->n_dd_groups = (ndd + kLanes - 1) / kLanes;
    p->n_dd_pad = p->n_dd_groups * kLanes;
    // polarized synthesis near the poles
    if (int rcp = build_pol_tables(p)) return rcp;

    // recurrence coefficients
    p->coef_off.resize(L + 2);
    p->coef_off[0] = 0;
    // runs start at even entries so that each (even, odd) entry pair the
    // kernel reads is one aligned 64-byte load
    for (int m = 0; m <= L; m++) {
        long long cnt = (L - m + 1) + kCoefPad;
        p->coef_off[m + 1] = p->coef_off[m] + cnt + (cnt & 1);
    }
    long long ne = p->coef_off[L + 1];
    ctx.coefl.assign(3 * (size_t)ne, 0.0L);
    p->coef_hi.assign(4 * (size_t)ne, 0.0);
    p->coef_lo.assign(4 * (size_t)ne, 0.0);
    parallel_for(L + 1, nth, coef_worker, &ctx);

    // chain start values
    p->start_idx.assign((size_t)(L + 1) * 2 * np, kDead);
    p->start_val.assign((size_t)(L + 1) * 2 * 2 * np, 0.0);
    p->start_lo.assign((size_t)(L + 1) * 2 * 2 * std::max(p->n_dd_pad, 1), 0.0);
    ctx.steps.assign(np, 0);
    ctx.alive.assign(np, 0);
    ctx.keep_ld = p->eps > 0.0 || p->opts.interp;
    if (ctx.keep_ld) ctx.start_ld.assign((size_t)(L + 1) * 2 * 2 * np, 0.0L);
    parallel_for(p->n_north, nth, start_worker, &ctx);
    if (ctx.bad.load())
        return fail(SHT_EUNSUPPORTED,
                    "a Legendre chain start value underflows double precision");
    p->n_step = p->n_step_exec = p->n_step_dd = 0;
    for (int k = 0; k < np; k++) {
        p->n_step += ctx.alive[k];
        p->n_step_exec += ctx.steps[k];
        if (k < p->n_dd_pad) p->n_step_dd += ctx.steps[k];
    }
    int ng = np / kLanes;
    p->grp_lo.assign((size_t)(L + 1) * ng, kDead);
    p->grp_hi.assign((size_t)(L + 1) * ng, -1);
    ctx.lane_steps.assign(L + 1, 0);
    parallel_for(L + 1, nth, group_worker, &ctx);
    p->n_step_lanes = 0;
    for (int m = 0; m <= L; m++) p->n_step_lanes += ctx.lane_steps[m];

    // ring FFT tables: twiddles, Bluestein sizes, LDS classes
    int maxS = 2;
    p->ring_M.assign(p->nrings, 0);
    p->ring_bs_off.assign(p->nrings, -1);
    p->ring_chirp_off.assign(p->nrings, 0);
    std::vector<long long> bs_of_n(4 * N + 1, -1), chirp_of_n(4 * N + 1, -1);
    BsCtx bctx;
    bctx.p = p;
    long long bs_total = 0, chirp_total = 0;
    for (int r = 0; r < p->nrings; r++) {
        int n = p->ring_J[r] / 2;
        if (is_pow2(n)) {
            maxS = std::max(maxS, n);
            continue;
        }
        // n = J/2 is even (J = 4i or 4 nside); the kernels split the DFT into
        // its even and odd halves and run Bluestein on length h = n/2
        const int h = n / 2;
        int M = 1 << ilog2(2LL * h - 1);
        p->ring_M[r] = M;
        maxS = std::max(maxS, M);
        if (bs_of_n[h] < 0) {
            bs_of_n[h] = bs_total;
            chirp_of_n[h] = chirp_total;
            bctx.ns.push_back(h);
            bctx.offs.push_back(bs_total);
            bctx.coffs.push_back(chirp_total);
            bs_total += M;
            chirp_total += h;
        }
        p->ring_bs_off[r] = bs_of_n[h];
        p->ring_chirp_off[r] = chirp_of_n[h];
    }
    if (maxS > 8192 || N > 2048)
        return fail(SHT_EUNSUPPORTED, "ring FFT larger than the kernels' limit (nside > 2048)");
    p->bs_table.assign(2 * (size_t)std::max(bs_total, 1LL), 0.0);
    p->chirp.assign(2 * (size_t)std::max(chirp_total, 1LL), 0.0);
    parallel_for((long)bctx.ns.size(), nth, bs_worker, &bctx);
    p->tw_log = std::max(1, ilog2(maxS));
    int half = 1 << (p->tw_log - 1);
    p->tw.resize(2 * (size_t)half);
    for (int k = 0; k < half; k++) {
        ld ang = 2.0L * kPi * (ld)k / (ld)(1 << p->tw_log);
        p->tw[2 * k] = (double)cosl(ang);
        p->tw[2 * k + 1] = (double)sinl(ang);
    }
    if (ctx.keep_ld) {
        std::vector<ld> z2l(p->n_north);
        for (int k = 0; k < p->n_north; k++) z2l[k] = ctx.zl[k] * ctx.zl[k];
        BflyInput in{ctx.coefl.data(), ctx.start_ld.data(), z2l.data()};
        if (p->eps > 0.0) {
            int rc = build_butterfly(p, in);
            if (rc != SHT_OK) return rc;
        }
        if (p->opts.interp) {
            int rc = build_interp(p, in);
            if (rc != SHT_OK) return rc;
        }
        std::vector<ld>().swap(ctx.start_ld);
    }
    const int class_size[4] = {1024, 2048, 4096, 8192};
    p->classes.clear();
    for (int ci = 0; ci < 4; ci++) {
        for (int wrap = 0; wrap < 2; wrap++) {
            RingClass rc;
            rc.lds_entries = class_size[ci];
            rc.wrap = wrap != 0;
            for (int r = 0; r < p->nrings; r++) {
                int S = p->ring_M[r] ? p->ring_M[r] : p->ring_J[r] / 2;
                int lo = ci == 0 ? 0 : class_size[ci - 1];
                bool w = p->ring_J[r] / 2 <= L;
                if (S > lo && S <= class_size[ci] && w == rc.wrap) rc.rings.push_back(r);
            }
            if (!rc.rings.empty()) p->classes.push_back(rc);
        }
    }
    return SHT_OK;
}

// ---------------------------------------------------------------------
// Device upload.
// ---------------------------------------------------------------------
template <typename T>
static hipError_t up(T **dst, const std::vector<T> &src, size_t *bytes) {
    size_t nb = std::max<size_t>(src.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)dst, nb);
    if (e != hipSuccess) return e;
    *bytes += nb;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

int upload_tables(sht_plan_s *p) {
    size_t b = 0;
    hipError_t e = hipSuccess;
#define UP(d, h) \
    if (e == hipSuccess) e = up(&p->d, p->h, &b)
    UP(d_z2_hi, z2_hi);
    UP(d_z2_lo, z2_lo);
    UP(d_ring_J, ring_J);
    UP(d_ring_s, ring_s);
    UP(d_ring_M, ring_M);
    UP(d_ring_off, ring_off);
    UP(d_ring_bs_off, ring_bs_off);
    UP(d_coef_off, coef_off);
    UP(d_coef_hi, coef_hi);
    UP(d_coef_lo, coef_lo);
    UP(d_start_idx, start_idx);
    UP(d_start_val, start_val);
    UP(d_start_lo, start_lo);
    UP(d_grp_lo, grp_lo);
    UP(d_grp_hi, grp_hi);
    UP(d_tw, tw);
    UP(d_bs_table, bs_table);
    UP(d_chirp, chirp);
    UP(d_ring_chirp_off, ring_chirp_off);
    UP(d_pol_ring, pol_ring);
    UP(d_pol_K, pol_K);
#undef UP
    for (auto &rc : p->classes)
        if (e == hipSuccess) e = up(&rc.d_rings, rc.rings, &b);
    if (p->ip.built) {
        InterpPlan &f = p->ip;
#define UPI(d, h) \
    if (e == hipSuccess) e = up(&p->d, f.h, &b)
        UPI(d_ip_node_off, node_off);
        UPI(d_ip_x_hi, x_hi);
        UPI(d_ip_x_lo, x_lo);
        UPI(d_ip_gam, gam);
        UPI(d_ip_lamN, lamN);
        UPI(d_ip_sub, sub);
        UPI(d_ip_lane, lane);
        UPI(d_ip_val, val);
        UPI(d_ip_dd_task, dd_task);
        UPI(d_ip_dd_lane, dd_lane);
        UPI(d_ip_dd_val, dd_val);
        UPI(d_ip_patch, patch);
#undef UPI
    }
    if (p->bf.built) {
        BflyPlan &f = p->bf;
#define UPB(d, h) \
    if (e == hipSuccess) e = up(&p->d, f.h, &b)
        UPB(d_bf_res_task, res_task);
        UPB(d_bf_res_sub, res_sub);
        UPB(d_bf_res_lane, res_lane);
        UPB(d_bf_res_val, res_val);
        UPB(d_bf_perm, perm);
        UPB(d_bf_node_i, node_i);
        UPB(d_bf_f1_unit, f1_unit);
        UPB(d_bf_l1_plain, l1_plain);
        UPB(d_bf_fold_slot, fold_slot);
        UPB(d_bf_T, T);
#undef UPB
        if (e == hipSuccess && p->opts.store_fp32) {
            const size_t n = std::max<size_t>(f.T.size(), 1);
            e = hipMalloc((void **)&p->d_bf_T32, n * sizeof(float));
            b += n * sizeof(float);
            std::vector<float> buf;
            const size_t chunk = (size_t)1 << 24;
            for (size_t o = 0; e == hipSuccess && o < f.T.size(); o += chunk) {
                const size_t cnt = std::min(chunk, f.T.size() - o);
                buf.resize(cnt);
                for (size_t i = 0; i < cnt; i++) buf[i] = (float)f.T[o + i];
                e = hipMemcpy(p->d_bf_T32 + o, buf.data(), cnt * sizeof(float), hipMemcpyHostToDevice);
            }
        }
        if (e == hipSuccess && p->opts.store_transpose)
            e = bf_store_transposed(p, f.T.size(), f.node_i.size() / kBfNodeInts, &b);
        // large interpolation data lives on the device only
        if (e == hipSuccess && f.T.size() * sizeof(double) > ((size_t)256 << 20)) {
            std::vector<double>().swap(f.T);
            f.host_T_kept = false;
        }
    }
    p->device_bytes = b;
    if (e != hipSuccess) {
        free_device_tables(p);
        return fail(e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EDEVICE,
                    std::string("plan upload: ") + hipGetErrorString(e));
    }
    return SHT_OK;
}

void free_device_tables(sht_plan_s *p) {
    void *ptrs[] = {p->d_z2_hi,     p->d_z2_lo,     p->d_ring_J,     p->d_ring_s,   p->d_ring_M,
                    p->d_ring_off,  p->d_ring_bs_off, p->d_coef_off, p->d_coef_hi,  p->d_coef_lo,
                    p->d_start_idx, p->d_start_val, p->d_start_lo,   p->d_grp_lo,   p->d_grp_hi,
                    p->d_tw,        p->d_bs_table,  p->d_chirp,      p->d_ring_chirp_off,
                    p->d_pol_ring,  p->d_pol_K,
                    p->d_bf_res_task, p->d_bf_res_lane, p->d_bf_res_sub,
                    p->d_bf_res_val, p->d_bf_T,      p->d_bf_T32,   p->d_bf_Tt,    p->d_bf_Tt32, p->d_bf_perm,
                    p->d_bf_node_i, p->d_bf_f1_unit, p->d_bf_l1_plain, p->d_bf_fold_slot,
                    p->d_ip_node_off, p->d_ip_x_hi, p->d_ip_x_lo, p->d_ip_gam, p->d_ip_lamN,
                    p->d_ip_sub, p->d_ip_lane, p->d_ip_val, p->d_ip_dd_task, p->d_ip_dd_lane, p->d_ip_dd_val,
                    p->d_ip_patch};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    for (auto &rc : p->classes)
        if (rc.d_rings) (void)hipFree(rc.d_rings), rc.d_rings = nullptr;

    p->d_z2_hi = p->d_z2_lo = nullptr;
    p->d_ring_J = p->d_ring_s = p->d_ring_M = nullptr;
    p->d_ring_off = p->d_ring_bs_off = p->d_coef_off = nullptr;
    p->d_coef_hi = p->d_coef_lo = nullptr;
    p->d_start_idx = nullptr;
    p->d_start_val = p->d_start_lo = nullptr;
    p->d_grp_lo = p->d_grp_hi = nullptr;
    p->d_tw = p->d_bs_table = p->d_chirp = nullptr;
    p->d_ring_chirp_off = nullptr;
    p->d_pol_ring = p->d_pol_K = nullptr;
    p->d_bf_res_task = p->d_bf_res_lane = p->d_bf_res_sub = nullptr;
    p->d_bf_res_val = p->d_bf_T = nullptr;
    p->d_bf_T32 = nullptr;
    p->d_bf_Tt = nullptr;
    p->d_bf_Tt32 = nullptr;
    p->d_bf_perm = nullptr;
    p->d_bf_node_i = nullptr;
    p->d_bf_f1_unit = p->d_bf_l1_plain = p->d_bf_fold_slot = nullptr;
    p->d_ip_node_off = nullptr;
    p->d_ip_x_hi = p->d_ip_x_lo = p->d_ip_gam = p->d_ip_lamN = p->d_ip_val = nullptr;
    p->d_ip_sub = p->d_ip_lane = p->d_ip_dd_task = p->d_ip_dd_lane = nullptr;
    p->d_ip_dd_val = nullptr;
    p->d_ip_patch = nullptr;
    p->device_bytes = 0;
}

}  // namespace sht
