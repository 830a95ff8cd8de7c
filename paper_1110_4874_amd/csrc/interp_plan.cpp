// Host precompute of the interpolation form of the Legendre phase (Sec. 3.3
// of the Wavemoth paper, Eq. 23): for order m and parity t the phase
//   q^t_m(z) = sum_{i<n} a_{m+t+2i} P~_{m+t+2i}^m(z)
// lies in the span of the chain functions (1 - z^2)^{m/2} z^t p_i(z^2),
// p_i a polynomial of degree i, so it is fixed by its values at n points.
// With N = m + t + 2n the function P~_N^m has exactly n roots z_j in (0, 1),
// and since P~_N^m(y) / (y^2 - z_j^2) lies in that span, vanishes at every
// other root and equals P~_N'(z_j) / (2 z_j) at z_j,
//   q^t_m(y) = P~_N^m(y) sum_j gamma_j q^t_m(z_j) / (y^2 - z_j^2),
//   gamma_j  = 2 z_j / P~_N'(z_j)
// exactly (the first barycentric form of Lagrange interpolation in x = z^2).
// The derivative at a root follows from
//   (1 - z^2) P~_l' = -l z P~_l + (2l + 1) a_l P~_{l-1},
// a_l = sqrt((l^2 - m^2)/(4 l^2 - 1)).  The roots x_j = z_j^2 are the
// eigenvalues of the chain's symmetric tridiagonal Jacobi matrix: the
// two-step recurrence of App. A.2 reads
//   z^2 P~_l = c_l P~_{l+2} + d_l P~_l + c_{l-2} P~_{l-2},
// so diagonal d_l and off-diagonal c_l for l = m + t + 2i, i < n.  They are
// found with the implicit QL iteration with Wilkinson shifts (Bowdler,
// Martin, Reinsch and Wilkinson, 1968), in long double.
//
// Precomputed per (m, t): the nodes x_j (double-double, so that the GPU forms
// y^2 - x_j without cancellation error when a ring falls close to a node),
// gamma_j, and the first node-chain values above the cutoff (App. A.2), laid
// out as tasks of the butterfly residual kernel so that the same kernel
// evaluates q at the nodes; per (m, t, north ring) the value P~_N^m(y_k)
// (zero where the ring's whole chain stays below the cutoff, where the
// brute-force path also writes zero).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cfloat>
#include <cstring>

#include "internal.h"

namespace sht {

typedef long double ld;

namespace {

ld a_one(int l, int m) {  // a_l of the one-step recurrence
    if (l <= m) return 0.0L;
    return sqrtl((ld)(l - m) * (ld)(l + m) / ((ld)(2 * l - 1) * (ld)(2 * l + 1)));
}

// Eigenvalues of the symmetric tridiagonal matrix with diagonal d[0..n) and
// off-diagonal e[0..n-1) (e[i] couples i and i + 1), returned ascending in d.
// Implicit QL with Wilkinson shifts and deflation on negligible off-diagonals.
bool tridiag_eigenvalues(std::vector<ld> &d, std::vector<ld> e) {
    const int n = (int)d.size();
    e.resize(n, 0.0L);
    const ld tiny = LDBL_EPSILON;
    for (int l = 0; l < n; l++) {
        for (int iter = 0;; iter++) {
            int m = l;
            for (; m < n - 1; m++) {
                const ld s = fabsl(d[m]) + fabsl(d[m + 1]);
                if (fabsl(e[m]) <= tiny * s) break;
            }
            if (m == l) break;
            if (iter > 60) return false;
            // shift: eigenvalue of the leading 2x2 block closer to d[l]
            ld g = (d[l + 1] - d[l]) / (2.0L * e[l]);
            ld r = hypotl(g, 1.0L);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            ld s = 1.0L, c = 1.0L, p = 0.0L;
            int i = m - 1;
            bool split = false;
            for (; i >= l; i--) {
                const ld f = s * e[i], b = c * e[i];
                r = hypotl(f, g);
                e[i + 1] = r;
                if (r == 0.0L) {  // an exact zero decouples the block
                    d[i + 1] -= p;
                    e[m] = 0.0L;
                    split = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0L * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
            }
            if (split) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0L;
        }
    }
    std::sort(d.begin(), d.end());
    return true;
}

struct IpCtx {
    sht_plan_s *p;
    const BflyInput *in;
    std::vector<long long> node_off;
    std::vector<ld> xl;                  // [nodes] roots
    std::vector<int> i0;                 // [nodes] first chain row above the cutoff (aligned)
    std::vector<double> v0, v1;          // [nodes] chain values at i0, i0 + 1
    std::vector<double> v0lo, v1lo;      // [nodes] their low parts (double-double)
    std::vector<double> gam;             // [nodes]
    std::vector<long long> steps;        // [(L+1)*2] node chain steps executed
    std::atomic<int> bad{0};
};

// Nodes, weights and chain starts of one (m, t).
void item_worker(long it, void *vctx) {
    IpCtx *c = (IpCtx *)vctx;
    const sht_plan_s *p = c->p;
    const int m = (int)(it / 2), t = (int)(it % 2), L = p->L;
    const int n = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
    if (n == 0) return;
    const long long base = c->node_off[it];
    // Jacobi matrix of the chain in x = z^2 (two-step recurrence, App. A.2)
    std::vector<ld> d(n), e(n > 1 ? n - 1 : 0);
    for (int i = 0; i < n; i++) {
        const int l = m + t + 2 * i;
        d[i] = a_one(l + 1, m) * a_one(l + 1, m) + a_one(l, m) * a_one(l, m);
        if (i + 1 < n) e[i] = a_one(l + 1, m) * a_one(l + 2, m);
    }
    if (!tridiag_eigenvalues(d, e)) {
        c->bad.store(1);
        return;
    }
    const int N = m + t + 2 * n;
    const ld cutoff = (ld)p->opts.cutoff;
    long long steps = 0;
    // a_l for l = m .. N (one-step recurrence), and the z-independent factor
    // of the sectoral value, sqrt((2m+1)/(4 pi) prod_{k<=m} (2k-1)/(2k)),
    // as mantissa * 2^cE
    std::vector<ld> al(N - m + 2);
    for (int l = m; l <= N + 1; l++) al[l - m] = a_one(l, m);
    ld cm = 1.0L;
    long cE = 0;
    int ex;
    for (int k = 1; k <= m; k++) {
        cm *= sqrtl((ld)(2 * k - 1) / (ld)(2 * k));
        cm = frexpl(cm, &ex);
        cE += ex;
    }
    cm *= sqrtl((ld)(2 * m + 1) / (4.0L * 3.14159265358979323846264338327950288L));
    if (m & 1) cm = -cm;
    for (int j = 0; j < n; j++) {
        const ld x = d[j];
        if (!(x > 0.0L && x < 1.0L)) {
            c->bad.store(1);
            return;
        }
        const ld z = sqrtl(x), st = sqrtl(1.0L - x);
        // sectoral value P~_m^m(z) = cm sin^m(theta), the power by repeated
        // squaring with exponent tracking
        ld mant = cm, pw = frexpl(st, &ex);
        long E = cE, bE = ex;
        for (int r = m; r > 0; r >>= 1) {
            if (r & 1) {
                mant = frexpl(mant * pw, &ex);
                E += ex + bE;
            }
            pw = frexpl(pw * pw, &ex);
            bE = 2 * bE + ex;
        }
        ld pm1 = 0.0L, p0 = mant;  // P~_{l-1}, P~_l (scaled by 2^-E), l = m
        int found = -1;
        ld s0 = 0, s1 = 0;
        long sE = 0;
        for (int l = m; l <= N; l++) {
            if (l > m) {  // advance to l
                const ld alv = al[l - m], alm1 = al[l - 1 - m];
                const ld pn = (z * p0 - alm1 * pm1) / alv;
                pm1 = p0;
                p0 = pn;
                const ld big = std::max(fabsl(p0), fabsl(pm1));
                if (big > 0x1p400L) {
                    p0 = ldexpl(p0, -400);
                    pm1 = ldexpl(pm1, -400);
                    E += 400;
                }
            }
            if (l == N) break;
            if (((l - m - t) & 1) == 0 && l >= m + t) {
                const int i = (l - m - t) / 2;  // chain index of l
                if (found < 0) {
                    if (i % kChunk == 0) {
                        s0 = p0;
                        sE = E;
                    }
                    if (i % kChunk == 1) s1 = ldexpl(p0, (int)(E - sE));
                    if (E > -16000 && fabsl(ldexpl(p0, (int)E)) >= cutoff) {
                        found = i - i % kChunk;
                        if (i % kChunk == 0) s1 = 0;  // set once the next chain value exists
                    }
                } else if (i == found + 1) {
                    s1 = ldexpl(p0, (int)(E - sE));
                }
            }
        }
        // here p0 = P~_N, pm1 = P~_{N-1} (scaled by 2^-E)
        const ld aN = al[N - m];
        const ld dscaled = (ld)(2 * N + 1) * aN * pm1 - (ld)N * z * p0;  // (1 - x) P~_N'(z) * 2^-E
        const ld g = 2.0L * z * (1.0L - x) / dscaled;
        const ld gam = ldexpl(g, (int)-E);
        const size_t q = (size_t)(base + j);
        c->xl[q] = x;
        c->gam[q] = (double)gam;
        if (!std::isfinite(c->gam[q]) || c->gam[q] == 0.0) c->bad.store(2);
        if (found >= 0) {
            c->i0[q] = found;
            const ld a0 = ldexpl(s0, (int)sE), a1 = ldexpl(s1, (int)sE);
            c->v0[q] = (double)a0;
            c->v1[q] = (double)a1;
            c->v0lo[q] = (double)(a0 - (ld)c->v0[q]);
            c->v1lo[q] = (double)(a1 - (ld)c->v1[q]);
            if (std::max(fabs(c->v0[q]), fabs(c->v1[q])) < 1e-290) c->bad.store(3);
            steps += n - found;
        } else {
            c->i0[q] = n;  // the whole chain stays below the cutoff: no work, output 0
            c->v0[q] = c->v1[q] = c->v0lo[q] = c->v1lo[q] = 0.0;
        }
    }
    c->steps[it] = steps;
}

// P~_N^m at every north ring for (m, t): the ring's chain continued from its
// stored start to chain index n (two-step recurrence in long double).
struct LamCtx {
    sht_plan_s *p;
    const BflyInput *in;
    std::vector<double> *out;
};

void lam_worker(long it, void *vctx) {
    LamCtx *c = (LamCtx *)vctx;
    const sht_plan_s *p = c->p;
    const int m = (int)(it / 2), t = (int)(it % 2), L = p->L, np = p->n_north_pad;
    const int n = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
    double *dst = c->out->data() + (size_t)it * np;
    if (n == 0) return;
    const ld *cf = c->in->coefl + 3 * p->coef_off[m];
    for (int k = 0; k < p->n_north; k++) {
        const int s = p->start_idx[(size_t)it * np + k];
        if (s >= kDead || s >= n) {
            dst[k] = 0.0;
            continue;
        }
        ld P0 = c->in->start_ld[((size_t)it * 2 + 0) * np + k];
        ld P1 = c->in->start_ld[((size_t)it * 2 + 1) * np + k];
        const ld z2 = c->in->z2l[k];
        // P0, P1: chain indices s, s + 1; advance until P0 is at index n
        for (int i = s; i < n; i++) {
            const int e = t + 2 * i + 2;  // coefficients producing chain index i + 2
            const ld P2 = (z2 * cf[3 * e] + cf[3 * e + 1]) * P1 + cf[3 * e + 2] * P0;
            P0 = P1;
            P1 = P2;
        }
        dst[k] = (double)P0;
    }
}

// Smallest |y^2 - x_j| below which a ring is evaluated directly: the nodes
// and P~_N(y) carry errors of a few 1e-19 in x, so elsewhere a term's
// relative error stays below ~5e-14.
constexpr long double kDirectGap = 1.5e-5L;

struct DirCtx {
    const sht_plan_s *p;
    const BflyInput *in;
    const IpCtx *c;
    std::vector<std::vector<int>> rings;  // [m] north rings evaluated directly, ascending
};

void direct_worker(long m, void *vctx) {
    DirCtx *dc = (DirCtx *)vctx;
    const sht_plan_s *p = dc->p;
    const IpCtx *c = dc->c;
    const int L = p->L, np = p->n_north_pad;
    for (int k = 0; k < p->n_north; k++) {
        const ld y2 = dc->in->z2l[k];
        bool near = false, any = false;
        for (int t = 0; t < 2 && !near; t++) {
            const long it = 2 * m + t;
            const int n = (L - (int)m - t >= 0) ? (L - (int)m - t) / 2 + 1 : 0;
            if (n == 0) continue;
            const int s0 = p->start_idx[(size_t)it * np + k];
            if (s0 >= kDead || s0 >= n) continue;  // dead chain: the value is 0 either way
            any = true;
            const ld *x = c->xl.data() + c->node_off[it];
            const ld *hi = std::lower_bound(x, x + n, y2);
            if (hi < x + n && *hi - y2 < kDirectGap) near = true;
            if (hi > x && y2 - hi[-1] < kDirectGap) near = true;
        }
        if (near && any) dc->rings[m].push_back(k);
    }
}

}  // namespace

int build_interp(sht_plan_s *p, const BflyInput &in) {
    auto t0 = std::chrono::steady_clock::now();
    const int L = p->L;
    InterpPlan &ip = p->ip;
    ip = InterpPlan();
    IpCtx c;
    c.p = p;
    c.in = &in;
    const long items = (long)(L + 1) * 2;
    c.node_off.assign(items + 1, 0);
    for (long it = 0; it < items; it++) {
        const int m = (int)(it / 2), t = (int)(it % 2);
        const int n = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
        c.node_off[it + 1] = c.node_off[it] + n;
    }
    const long long nodes = c.node_off[items];
    c.xl.assign(nodes, 0.0L);
    c.i0.assign(nodes, 0);
    c.v0.assign(nodes, 0.0);
    c.v1.assign(nodes, 0.0);
    c.v0lo.assign(nodes, 0.0);
    c.v1lo.assign(nodes, 0.0);
    c.gam.assign(nodes, 0.0);
    c.steps.assign(items, 0);
    parallel_for(items, p->opts.nthreads, item_worker, &c);
    if (c.bad.load()) return fail(SHT_EUNSUPPORTED, "interpolation nodes or weights out of double range");
    // Rings closer to a node of their order than the nodes' own precision
    // allows for.  The roots come from a long-double eigenvalue iteration,
    // good to a few 1e-19 in x, and P~_N(y) is the long-double chain value;
    // in the term of node j both are off by that much against y^2 - x_j, so
    // a ring within kDirectGap of a node of either parity is evaluated at
    // the ring itself instead (both parities), like a node: 1-2 percent of
    // the (order, ring) pairs at L ~ 4096.
    DirCtx dc{p, &in, &c, {}};
    dc.rings.resize(L + 1);
    parallel_for(L + 1, p->opts.nthreads, direct_worker, &dc);
    const int np = p->n_north_pad;
    auto live = [&](long it, int k, int n) {
        const int s0 = p->start_idx[(size_t)it * np + k];
        return s0 < kDead && s0 < n;
    };
    // new layout: the n nodes of (m, t), then its direct rings, x ascending
    std::vector<long long> off(items + 1, 0);
    for (long it = 0; it < items; it++) {
        const int m = (int)(it / 2), t = (int)(it % 2);
        const int n = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
        long long d = 0;
        for (int k : dc.rings[m])
            if (live(it, k, n)) d++;
        off[it + 1] = off[it] + n + d;
    }
    const long long total = off[items];
    if (total > 0x7fffffffLL) return fail(SHT_EUNSUPPORTED, "interpolation tables exceed 32-bit offsets");
    // every point: x (long double), first chain row, start values
    struct Pt {
        ld x;
        int i0;
        double v0, v0lo, v1, v1lo, gam;
    };
    std::vector<Pt> pts(total);
    for (long it = 0; it < items; it++) {
        const int m = (int)(it / 2), t = (int)(it % 2);
        const int n = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
        const long long b0 = c.node_off[it], nb0 = off[it];
        for (int j = 0; j < n; j++) {
            const long long q = b0 + j;
            pts[nb0 + j] = {c.xl[q], c.i0[q], c.v0[q], c.v0lo[q], c.v1[q], c.v1lo[q], c.gam[q]};
        }
        long long d = nb0 + n;
        for (auto r = dc.rings[m].rbegin(); r != dc.rings[m].rend(); ++r) {  // x ascending
            const int k = *r;
            if (!live(it, k, n)) continue;
            const ld a0 = in.start_ld[((size_t)it * 2 + 0) * np + k], a1 = in.start_ld[((size_t)it * 2 + 1) * np + k];
            const double h0 = (double)a0, h1 = (double)a1;
            pts[d++] = {in.z2l[k], p->start_idx[(size_t)it * np + k], h0, (double)(a0 - (ld)h0), h1,
                        (double)(a1 - (ld)h1), 0.0};
        }
    }
    for (int m = 0; m <= L; m++)
        for (int k : dc.rings[m]) {
            int slot[2] = {-1, -1};
            for (int t = 0; t < 2; t++) {
                const long it = 2L * m + t;
                const int n = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
                if (!live(it, k, n)) continue;
                // position of ring k among the live direct rings of (m, t), x ascending
                long long pos = 0;
                for (int k2 : dc.rings[m])
                    if (k2 > k && live(it, k2, n)) pos++;
                slot[t] = (int)(off[it] + n + pos);
            }
            if (slot[0] < 0 && slot[1] < 0) continue;
            ip.patch.insert(ip.patch.end(), {m, k, slot[0], slot[1]});
            ip.direct += (slot[0] >= 0) + (slot[1] >= 0);
        }
    ip.node_off = off;
    ip.x_hi.resize(total);
    ip.x_lo.resize(total);
    ip.gam.resize(total);
    for (long long q = 0; q < total; q++) {
        ip.x_hi[q] = (double)pts[q].x;
        ip.x_lo[q] = (double)(pts[q].x - (ld)ip.x_hi[q]);
        ip.gam[q] = pts[q].gam;
    }
    ip.nodes = total;
    for (long it = 0; it < items; it++) ip.steps += c.steps[it];
    // node tasks in the residual kernel's format: pieces of up to
    // kBfPieceRings points of one (m, t); the points nearest the pole (the
    // largest x, at the end of each group) whose sin(theta) is below the
    // plan's double-double threshold get compensated one-wave tasks instead,
    // three times the brute-force path's band: a node's error reaches every
    // ring through the interpolation weights, so the polar nodes' FP64 error
    // (~l eps / sin(theta)) is held three times lower than on the rings
    const double dd_sin = 3.0 * (p->opts.dd_sin < 0 ? 0.1 * (double)L / 4095.0 : p->opts.dd_sin);
    const ld x_dd = 1.0L - (ld)dd_sin * (ld)dd_sin;
    for (long it = 0; it < items; it++) {
        const int m = (int)(it / 2), t = (int)(it % 2);
        const int n = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
        // two groups, each x ascending: the nodes, then the direct rings
        const long long groups[2][2] = {{off[it], off[it] + n}, {off[it] + n, off[it + 1]}};
        for (int gi = 0; gi < 2; gi++) {
            const long long g0 = groups[gi][0], g1 = groups[gi][1];
            long long gfp = g1;  // points [g0, gfp) run in FP64, [gfp, g1) compensated
            while (gfp > g0 && pts[gfp - 1].x > x_dd) gfp--;
            if (gi == 1)
                for (long long q = g0; q < g1; q++) ip.steps += n - std::min(n, pts[q].i0);
            for (long long j0 = gfp; j0 < g1; j0 += 64) {
                const int nl = (int)std::min<long long>(64, g1 - j0);
                int imin = n;
                for (int j = 0; j < nl; j++) imin = std::min(imin, pts[j0 + j].i0);
                const long long lane0 = (long long)ip.dd_lane.size() / 2;
                if (lane0 > 0x7fffffffLL) return fail(SHT_EUNSUPPORTED, "interpolation tables exceed 32-bit offsets");
                ip.dd_task.insert(ip.dd_task.end(), {t, m, n, nl, (int)j0, (int)lane0, imin, 0});
                for (int j = 0; j < 64; j++) {
                    const Pt &q = pts[j0 + std::min(j, nl - 1)];
                    ip.dd_lane.insert(ip.dd_lane.end(), {(int)(j0 + std::min(j, nl - 1)), j < nl ? q.i0 : INT32_MAX});
                    ip.dd_val.insert(ip.dd_val.end(), {q.v0, q.v0lo, q.v1, q.v1lo});
                }
                ip.dd_nodes += nl;
            }
            for (long long j0 = g0; j0 < gfp; j0 += kBfPieceRings) {
                const int nl = (int)std::min<long long>(kBfPieceRings, gfp - j0);
                int imin = n;
                for (int j = 0; j < nl; j++) imin = std::min(imin, pts[j0 + j].i0);
                const long long lane0 = (long long)ip.lane.size() / 2;
                if (lane0 > 0x7fffffffLL) return fail(SHT_EUNSUPPORTED, "interpolation tables exceed 32-bit offsets");
                ip.sub.insert(ip.sub.end(), {t, imin, n, nl, (int)j0, m, (int)lane0, 0});
                for (int j = 0; j < kBfPieceRings; j++) {
                    if (j < nl) {
                        ip.lane.insert(ip.lane.end(), {(int)(j0 + j), pts[j0 + j].i0});
                        ip.val.push_back(pts[j0 + j].v0);
                        ip.val.push_back(pts[j0 + j].v1);
                    } else {
                        ip.lane.insert(ip.lane.end(), {0, INT32_MAX});
                        ip.val.push_back(0.0);
                        ip.val.push_back(0.0);
                    }
                }
                ip.exec += (long long)(n - imin) * kBfPieceRings;
            }
        }
    }
    // P~_N on the rings
    ip.lamN.assign((size_t)items * p->n_north_pad, 0.0);
    LamCtx lc{p, &in, &ip.lamN};
    parallel_for(items, p->opts.nthreads, lam_worker, &lc);
    ip.built = 1;
    ip.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return SHT_OK;
}

// Host evaluation of q^t_m at the north rings through the nodes, as the GPU
// does it (node chains in double from the stored starts, then Eq. 23 with
// double-double differences).  x: n_t real coefficients; y: n_north values.
int interp_apply_host(const sht_plan_s *p, int m, int t, const double *x, double *y) {
    const InterpPlan &ip = p->ip;
    const int L = p->L, np = p->n_north_pad;
    const int n = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
    const long it = 2L * m + t;
    const long long b0 = ip.node_off[it];
    std::vector<double> Q((size_t)(ip.node_off[it + 1] - b0), 0.0);  // the nodes, then the direct rings
    const double *cf = p->coef_hi.data() + 4 * p->coef_off[m];
    // node values: the pieces of this (m, t)
    for (size_t s = 0; s < ip.sub.size(); s += 8) {
        const int *h = &ip.sub[s];
        if (h[5] != m || h[0] != t) continue;
        for (int j = 0; j < h[3]; j++) {
            const size_t li = (size_t)h[6] + j;
            const int q = ip.lane[2 * li], i0 = ip.lane[2 * li + 1];
            double P0 = ip.val[2 * li], P1 = ip.val[2 * li + 1], acc = 0.0;
            const double z2 = ip.x_hi[q];
            for (int i = i0; i < n; i++) {
                acc += P0 * x[i];
                const double *e = cf + 4 * (t + 2 * i + 2);
                const double P2 = (z2 * e[0] + e[1]) * P1 + e[2] * P0;
                P0 = P1;
                P1 = P2;
            }
            Q[q - b0] = acc;
        }
    }
    // compensated nodes: the chain in long double (the GPU uses double-double)
    for (size_t s = 0; s < ip.dd_task.size(); s += 8) {
        const int *h = &ip.dd_task[s];
        if (h[1] != m || h[0] != t) continue;
        for (int j = 0; j < h[3]; j++) {
            const size_t li = (size_t)h[5] + j;
            const int q = ip.dd_lane[2 * li], i0 = ip.dd_lane[2 * li + 1];
            const double *v = &ip.dd_val[4 * li];
            long double P0 = (long double)v[0] + v[1], P1 = (long double)v[2] + v[3], acc = 0.0L;
            const long double z2 = (long double)ip.x_hi[q] + ip.x_lo[q];
            const double *ch = p->coef_hi.data() + 4 * p->coef_off[m];
            const double *cl = p->coef_lo.data() + 4 * p->coef_off[m];
            for (int i = i0; i < n; i++) {
                acc += P0 * x[i];
                const int e = t + 2 * i + 2;
                const long double B = (long double)ch[4 * e] + cl[4 * e], AB = (long double)ch[4 * e + 1] + cl[4 * e + 1],
                                  G = (long double)ch[4 * e + 2] + cl[4 * e + 2];
                const long double P2 = (z2 * B + AB) * P1 + G * P0;
                P0 = P1;
                P1 = P2;
            }
            Q[q - b0] = (double)acc;
        }
    }
    for (int k = 0; k < p->n_north; k++) {
        const double lam = ip.lamN[(size_t)it * np + k];
        if (lam == 0.0) {
            y[k] = 0.0;
            continue;
        }
        double s = 0.0;
        for (int j = 0; j < n; j++) {
            double dd = (p->z2_hi[k] - ip.x_hi[b0 + j]) + (p->z2_lo[k] - ip.x_lo[b0 + j]);
            if (fabs(dd) < 1e-200) dd = dd < 0 ? -1e-200 : 1e-200;
            s += ip.gam[b0 + j] * Q[j] / dd;
        }
        y[k] = lam * s;
    }
    // rings evaluated directly
    for (size_t i = 0; i < ip.patch.size(); i += 4) {
        if (ip.patch[i] != m) continue;
        const int slot = ip.patch[i + 2 + t];
        y[ip.patch[i + 1]] = slot >= 0 ? Q[slot - b0] : 0.0;
    }
    return SHT_OK;
}

}  // namespace sht
