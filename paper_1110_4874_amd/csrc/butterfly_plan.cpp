// Host precompute of the butterfly-compressed Legendre operator (Sec. 3 of
// the Wavemoth paper), and its flattening into the records the GPU kernel
// walks.
//
// For each order m and parity t the matrix Lambda (rows: l = m + t + 2i,
// i = 0..n-1; columns: the north rings z_k) is factored as in Sec. 3.2,
// Eq. 21: Lambda = R S_d P_{d-1} ... P_1 S_1.  Level 1 splits the rows in
// two and takes the interpolative decomposition (Sec. 3.1, Eq. 19) of every
// (row half, column block of about `chunk` rings); level i > 1 joins the
// skeleton columns that two neighbouring level-(i-1) column groups kept in
// the same parent row block, splits the rows again and takes the ID of each
// half (Eq. 18).  After d levels the residual R consists of, per leaf (row
// block, column group), the Legendre values at the leaf's rows and its
// skeleton rings; the kernel regenerates those with the recurrence from two
// stored values per column (Sec. 3.4), so only the interpolation matrices
// (their dense, non-identity part, App. A.1) are streamed from memory.
//
// The depth d of each (m, t) minimises rho * (stored interpolation entries)
// + (residual recurrence elements), the paper's CPU/memory trade-off of
// Sec. 3.4 with rho set for MI355X instead of a CPU.
//
// Interpolative decomposition: Householder QR with column pivoting
// (Businger-Golub), stopped when the largest remaining column norm falls
// to eps * |R_11|; the interpolation matrix is [I | R_11^{-1} R_12] in
// pivoted column order.  Ties in the pivot choice go to the lowest column,
// so plans are deterministic.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace sht {

// ---------------------------------------------------------------------
// Interpolative decomposition of A (r x c, column-major, lda = r; A is
// overwritten).  Returns the rank k, the pivot order (piv[0..k) are the
// skeleton columns) and T (k x (c-k), row-major) with
// A[:, piv[k + j]] ~= sum_s A[:, piv[s]] T[s][j].
// ---------------------------------------------------------------------
int interp_decomp(double *A, int r, int c, double tol, double abs_floor, std::vector<int> &piv,
                  std::vector<double> &T) {
    piv.resize(c);
    std::iota(piv.begin(), piv.end(), 0);
    T.clear();
    if (r <= 0 || c <= 0) return 0;
    std::vector<double> vn1(c), vn2(c);
    for (int j = 0; j < c; j++) {
        const double *col = A + (size_t)j * r;
        double s = 0;
        for (int i = 0; i < r; i++) s += col[i] * col[i];
        vn1[j] = vn2[j] = std::sqrt(s);
    }
    const int kmax = std::min(r, c);
    const double tol3z = std::sqrt(2.220446049250313e-16);
    double r11 = 0;
    int k = 0;
    std::vector<double> v(r);
    for (int j = 0; j < kmax; j++) {
        int p = j;
        for (int q = j + 1; q < c; q++)
            if (vn1[q] > vn1[p]) p = q;
        if (j == 0) {
            r11 = vn1[p];
            if (!(r11 > abs_floor)) return 0;
        }
        if (vn1[p] <= tol * r11) break;
        if (p != j) {
            std::swap_ranges(A + (size_t)p * r, A + (size_t)p * r + r, A + (size_t)j * r);
            std::swap(piv[p], piv[j]);
            std::swap(vn1[p], vn1[j]);
            std::swap(vn2[p], vn2[j]);
        }
        // Householder reflector for A[j:, j]
        double *cj = A + (size_t)j * r;
        double alpha = cj[j], xn = 0;
        for (int i = j + 1; i < r; i++) xn += cj[i] * cj[i];
        xn = std::sqrt(xn);
        double tau = 0.0;
        if (xn != 0.0) {
            double beta = -std::copysign(std::hypot(alpha, xn), alpha);
            tau = (beta - alpha) / beta;
            double sc = 1.0 / (alpha - beta);
            v[j] = 1.0;
            for (int i = j + 1; i < r; i++) v[i] = cj[i] * sc;
            cj[j] = beta;
            for (int i = j + 1; i < r; i++) cj[i] = 0.0;
        }
        if (tau != 0.0) {
            // apply the reflector to the remaining columns, NW at a time: each
            // column's product with v is summed in row order as for a single
            // column, the NW sums interleaved (independent chains)
            constexpr int NW = 8;
            int q = j + 1;
            for (; q + NW <= c; q += NW) {
                double *cc[NW], w[NW];
                for (int u = 0; u < NW; u++) {
                    cc[u] = A + (size_t)(q + u) * r;
                    w[u] = cc[u][j];
                }
                for (int i = j + 1; i < r; i++) {
                    const double vi = v[i];
                    for (int u = 0; u < NW; u++) w[u] += vi * cc[u][i];
                }
                for (int u = 0; u < NW; u++) {
                    const double wu = w[u] * tau;
                    double *cq = cc[u];
                    cq[j] -= wu;
                    for (int i = j + 1; i < r; i++) cq[i] -= wu * v[i];
                }
            }
            for (; q < c; q++) {
                double *cq = A + (size_t)q * r;
                double w = cq[j];
                for (int i = j + 1; i < r; i++) w += v[i] * cq[i];
                w *= tau;
                cq[j] -= w;
                for (int i = j + 1; i < r; i++) cq[i] -= w * v[i];
            }
        }
        // downdate the remaining column norms, recomputing a norm once the
        // downdated ratio falls below sqrt(eps) (the cancellation safeguard of
        // Drmac and Bujanovic, 2008)
        for (int q = j + 1; q < c; q++) {
            if (vn1[q] == 0.0) continue;
            double *cq = A + (size_t)q * r;
            double t = std::fabs(cq[j]) / vn1[q];
            t = std::max(0.0, (1.0 + t) * (1.0 - t));
            double t2 = t * (vn1[q] / vn2[q]) * (vn1[q] / vn2[q]);
            if (t2 <= tol3z) {
                double s = 0;
                for (int i = j + 1; i < r; i++) s += cq[i] * cq[i];
                vn1[q] = vn2[q] = std::sqrt(s);
            } else {
                vn1[q] *= std::sqrt(t);
            }
        }
        k = j + 1;
    }
    // T = R11^{-1} R12 by back substitution along contiguous rows of T (R11
    // copied row-major); every entry is reduced over s2 = s+1 .. k-1 in
    // increasing order, as a column-by-column solve would
    const int nd = c - k;
    T.assign((size_t)k * nd, 0.0);
    std::vector<double> R((size_t)k * k);
    for (int s = 0; s < k; s++)
        for (int s2 = s; s2 < k; s2++) R[(size_t)s * k + s2] = A[(size_t)s2 * r + s];
    for (int s = k - 1; s >= 0; s--) {
        double *ts = T.data() + (size_t)s * nd;
        for (int d = 0; d < nd; d++) ts[d] = A[(size_t)(k + d) * r + s];
        for (int s2 = s + 1; s2 < k; s2++) {
            const double a = R[(size_t)s * k + s2];
            const double *t2 = T.data() + (size_t)s2 * nd;
            for (int d = 0; d < nd; d++) ts[d] -= a * t2[d];
        }
        const double diag = R[(size_t)s * k + s];
        for (int d = 0; d < nd; d++) ts[d] /= diag;
    }
    return k;
}

namespace {

// One ID block of the factorization.  Its columns C are given in order;
// skel holds the positions (ascending) of the skeleton columns inside C and
// code[c] is s >= 0 for the s-th skeleton column or -1-d for the d-th
// remaining (dense) column; T is k x (n - k), row-major [s][d].
struct Node {
    int k = 0, n = 0;
    std::vector<int> cols;   // ring index of each column of C
    std::vector<int> skel;   // ring index of each skeleton column, in order
    std::vector<int> code;   // [n]
    std::vector<double> T;   // [k][n-k]
};

struct Item {
    int n = 0;      // rows
    int depth = 0;  // levels kept
    int p2 = 1;     // column blocks at level 1
    std::vector<int> colb;                 // [p2+1] column block bounds
    std::vector<std::vector<Node>> lv;     // lv[i-1]: level i, index rho * G_i + gamma
    std::vector<int> st;                   // [K] first chain index run per ring (n if dead)
    // residual lanes, leaf by leaf: ring, first and end chain index, output
    // position inside the leaf level's vector (or ring for depth 0), and the
    // Legendre values at the first two chain indices
    std::vector<int> lane;                 // [nl][4]
    std::vector<double> lval;              // [nl][2]
    std::vector<int> seg;                  // [nseg][4] lane range and rows of each row block
    long long T_entries = 0, res_elems = 0;
};

int groups_at(const Item &it, int i) { return it.p2 >> (i - 1); }

void row_bounds(int n, int i, int rho, int *r0, int *r1) {
    int a = 0, b = n;
    for (int lv = i - 1; lv >= 0; lv--) {
        int mid = a + (b - a) / 2;
        if ((rho >> lv) & 1)
            a = mid;
        else
            b = mid;
    }
    *r0 = a;
    *r1 = b;
}

struct BfCtx {
    sht_plan_s *p;
    const BflyInput *in;
    std::vector<Item> items;  // [(L+1)*2]
    double eps_id, rho;
    int chunk, max_levels;
};

long long leaf_elems(const Item &it, int r0, int r1, const std::vector<int> &rings) {
    long long e = 0;
    for (int k : rings) e += std::max(0, r1 - std::max(r0, it.st[k]));
    return e;
}

void item_worker(long idx, void *vctx) {
    BfCtx *c = (BfCtx *)vctx;
    sht_plan_s *p = c->p;
    const int m = (int)(idx / 2), t = (int)(idx % 2);
    const int L = p->L, K = p->n_north, np = p->n_north_pad;
    Item &it = c->items[idx];
    const int n = (L - m - t >= 0) ? (L - m - t) / 2 + 1 : 0;
    it.n = n;
    it.st.assign(K, n);
    // columns of Lambda from the long-double chain starts
    const size_t row = (size_t)(2 * m + t);
    for (int k = 0; k < K; k++) {
        int s = p->start_idx[row * np + k];
        if (s < n) it.st[k] = s;
    }
    // column blocks: the largest power of two 2^pe with K / 2^pe >= chunk
    int pe = 0;
    while ((K >> (pe + 1)) >= c->chunk) pe++;
    it.p2 = 1 << pe;
    it.colb.resize(it.p2 + 1);
    for (int j = 0; j <= it.p2; j++) it.colb[j] = (int)((long long)j * K / it.p2);
    long long brute = 0;
    for (int k = 0; k < K; k++) brute += n - it.st[k];
    it.res_elems = brute;
    it.depth = 0;
    int maxd = pe + 1;
    while (maxd > 0 && (n >> maxd) < 4) maxd--;  // leaves keep >= 4 rows
    if (c->max_levels >= 0) maxd = std::min(maxd, c->max_levels);
    if (maxd == 0 || n == 0) {
        // brute force: one lane per ring from its chain start
        it.seg.insert(it.seg.end(), {0, K, 0, n});
        for (int k = 0; k < K; k++) {
            const int i0 = it.st[k];
            it.lane.insert(it.lane.end(), {k, i0, n, k});
            double a0 = 0, a1 = 0;
            if (i0 < n) {
                a0 = (double)c->in->start_ld[(row * 2 + 0) * np + k];
                a1 = (double)c->in->start_ld[(row * 2 + 1) * np + k];
            }
            it.lval.push_back(a0);
            it.lval.push_back(a1);
        }
        return;
    }

    std::vector<double> lam((size_t)K * n, 0.0);
    double amax = 0.0;
    {
        const long double *cf = c->in->coefl + 3 * p->coef_off[m];
        for (int k = 0; k < K; k++) {
            int s = it.st[k];
            if (s >= n) continue;
            const long double z2 = c->in->z2l[k];
            long double P0 = c->in->start_ld[(row * 2 + 0) * np + k];
            long double P1 = c->in->start_ld[(row * 2 + 1) * np + k];
            double *col = lam.data() + (size_t)k * n;
            for (int i = s; i < n; i++) {
                col[i] = (double)P0;
                amax = std::max(amax, std::fabs(col[i]));
                int e = t + 2 * i + 2;
                long double P2 = (z2 * cf[3 * e] + cf[3 * e + 1]) * P1 + cf[3 * e + 2] * P0;
                P0 = P1;
                P1 = P2;
            }
        }
    }
    const double floor_abs = 1e-30 * amax;

    std::vector<double> A;
    std::vector<int> piv;
    double best = (double)brute;
    long long Tsum = 0;
    for (int i = 1; i <= maxd; i++) {
        const int G = groups_at(it, i), nr = 1 << i;
        std::vector<Node> nodes((size_t)nr * G);
        long long lvT = 0, res = 0;
        for (int rho = 0; rho < nr; rho++) {
            int r0, r1;
            row_bounds(n, i, rho, &r0, &r1);
            const int rr = r1 - r0;
            for (int g = 0; g < G; g++) {
                Node &nd = nodes[(size_t)rho * G + g];
                if (i == 1) {
                    for (int k = it.colb[g]; k < it.colb[g + 1]; k++) nd.cols.push_back(k);
                } else {
                    const int Gp = groups_at(it, i - 1), pi = rho >> 1;
                    const Node &a = it.lv[i - 2][(size_t)pi * Gp + 2 * g];
                    const Node &b = it.lv[i - 2][(size_t)pi * Gp + 2 * g + 1];
                    nd.cols = a.skel;
                    nd.cols.insert(nd.cols.end(), b.skel.begin(), b.skel.end());
                }
                nd.n = (int)nd.cols.size();
                A.assign((size_t)rr * nd.n, 0.0);
                for (int q = 0; q < nd.n; q++)
                    std::memcpy(A.data() + (size_t)q * rr, lam.data() + (size_t)nd.cols[q] * n + r0,
                                sizeof(double) * rr);
                std::vector<double> Tp;
                nd.k = interp_decomp(A.data(), rr, nd.n, c->eps_id, floor_abs, piv, Tp);
                // skeleton in ascending column position; T rows follow
                std::vector<int> order(piv.begin(), piv.begin() + nd.k);
                std::vector<int> rank_of(nd.k);
                std::vector<int> sorted = order;
                std::sort(sorted.begin(), sorted.end());
                for (int s = 0; s < nd.k; s++)
                    rank_of[s] = (int)(std::lower_bound(sorted.begin(), sorted.end(), order[s]) - sorted.begin());
                std::vector<int> dense(piv.begin() + nd.k, piv.end());
                std::vector<int> dsorted = dense;
                std::sort(dsorted.begin(), dsorted.end());
                const int ndn = nd.n - nd.k;
                nd.code.assign(nd.n, 0);
                nd.skel.resize(nd.k);
                for (int s = 0; s < nd.k; s++) {
                    nd.code[sorted[s]] = s;
                    nd.skel[s] = nd.cols[sorted[s]];
                }
                for (int d = 0; d < ndn; d++) nd.code[dsorted[d]] = -1 - d;
                nd.T.assign((size_t)nd.k * ndn, 0.0);
                for (int s = 0; s < nd.k; s++)
                    for (int d = 0; d < ndn; d++) {
                        int dpos = (int)(std::lower_bound(dsorted.begin(), dsorted.end(), dense[d]) - dsorted.begin());
                        nd.T[(size_t)rank_of[s] * ndn + dpos] = Tp[(size_t)s * ndn + d];
                    }
                lvT += (long long)nd.k * ndn;
                res += leaf_elems(it, r0, r1, nd.skel);
            }
        }
        it.lv.push_back(std::move(nodes));
        Tsum += lvT;
        const double cost = c->rho * (double)Tsum + (double)res;
        if (c->max_levels >= 0) {  // forced depth
            it.depth = i;
            it.T_entries = Tsum;
            it.res_elems = res;
            continue;
        }
        if (cost < best) {
            best = cost;
            it.depth = i;
            it.T_entries = Tsum;
            it.res_elems = res;
        } else {
            break;  // the cost stopped falling
        }
    }
    it.lv.resize(it.depth);
    // residual lanes with their start values (from the long-double columns)
    auto lane = [&](int k, int r0, int r1, int out) {
        int i0 = std::min(std::max(r0, it.st[k]), r1);
        it.lane.insert(it.lane.end(), {k, i0, r1, out});
        const double *col = lam.data() + (size_t)k * n;
        it.lval.push_back(i0 < r1 ? col[i0] : 0.0);
        it.lval.push_back(i0 + 1 < n ? col[i0 + 1] : 0.0);
    };
    if (it.depth == 0) {
        it.seg.insert(it.seg.end(), {0, K, 0, n});
        for (int k = 0; k < K; k++) lane(k, 0, n, k);
    } else {
        const int d = it.depth, G = groups_at(it, d);
        int off = 0;
        for (int rho = 0; rho < (1 << d); rho++) {
            int r0, r1;
            row_bounds(n, d, rho, &r0, &r1);
            const int l0 = (int)it.lane.size() / 4;
            for (int g = 0; g < G; g++) {
                const Node &nd = it.lv[d - 1][(size_t)rho * G + g];
                for (int s = 0; s < nd.k; s++) lane(nd.skel[s], r0, r1, off + s);
                off += nd.k;
            }
            it.seg.insert(it.seg.end(), {l0, (int)it.lane.size() / 4, r0, r1});
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------
// Build every (m, t) tree and flatten them (both parities of one m share a
// work item of the kernel; see butterfly.hip for the record formats).
// ---------------------------------------------------------------------
int build_butterfly(sht_plan_s *p, const BflyInput &in) {
    auto t0 = std::chrono::steady_clock::now();
    const int L = p->L, K = p->n_north;
    BfCtx c;
    c.p = p;
    c.in = &in;
    c.items.resize((size_t)(L + 1) * 2);
    // IDs at eps / 4 by default: the transpose of the compressed operator
    // (the adjoint) applied to white-noise maps reached 1.7 eps with blocks
    // truncated at eps, and still 1.1 eps at eps / 2 once 21 maps were
    // sampled (L = 200, eps = 1e-10, three levels); eps / 4 keeps both
    // directions within eps there for ~2% fewer levels kept by the cost model.
    c.eps_id = p->eps / (p->opts.id_safety > 0 ? std::max(1.0, p->opts.id_safety) : 4.0);
    // rho 4 by default: at L = 4095, nside = 2048, 4 maps the FP64 level
    // launches stream an entry in the time of about 4 residual elements
    // (synthesis 11.92 / 11.47 / 11.67 ms at rho 2.5 / 4 / 6)
    c.rho = p->opts.rho > 0 ? p->opts.rho : 4.0;
    c.chunk = p->opts.chunk > 0 ? p->opts.chunk : 64;
    c.max_levels = p->opts.max_levels;
    parallel_for((long)c.items.size(), p->opts.nthreads, item_worker, &c);

    BflyPlan &b = p->bf;
    b = BflyPlan();
    b.K = K;
    {
        size_t nT = 0, ntask = 0;
        for (auto &it : c.items) {
            nT += (size_t)it.T_entries;
            for (size_t q = 0; q + 3 < it.seg.size(); q += 4)
                ntask += (size_t)(it.seg[q + 1] - it.seg[q] + kBfTaskRings - 1) / kBfTaskRings;
        }
        b.T.reserve(nT);
        b.res_task.reserve(8 * ntask);
        b.res_lane.reserve(2 * kBfTaskRings * ntask);
        b.res_val.reserve(2 * kBfTaskRings * ntask);
    }
    b.depth.assign((size_t)(L + 1) * 2, 0);
    // Vector regions of the workspace (entries of 2B values): Q holds the
    // level-1 output q^t of every (m, t) (or the residual output at depth 0),
    // LEAF the residual output at the deepest level kept, and R0 / R1 the
    // vectors that level launches produce for even / odd levels.  Offsets
    // are region-relative while building and made absolute at the end.
    enum { RQ = 0, RLEAF = 1, RR0 = 2, RR1 = 3 };
    // Orders may be processed in batches (order m goes to batch m mod nb)
    // whose live vectors fit a cache budget: each batch runs the residual,
    // the level launches and the fold before the next one starts.
    std::vector<long long> item_leaf(c.items.size(), 0), item_lvl((size_t)c.items.size() * (kBfMaxLv + 1), 0);
    for (size_t q = 0; q < c.items.size(); q++) {
        const Item &it = c.items[q];
        for (int i = 1; i <= it.depth; i++) {
            long long sz = 0;
            for (const Node &nd : it.lv[i - 1]) sz += nd.k;
            if (i == it.depth)
                item_leaf[q] = sz;
            else
                item_lvl[q * (kBfMaxLv + 1) + i] = sz;
        }
    }
    // (batch_mib = 0: one batch; measured faster on MI355X, where the level
    // launches need every order's nodes in flight more than cache residency)
    const double target = p->opts.batch_mib > 0 ? p->opts.batch_mib * 1048576.0 : 1e300;  // at 8 doubles per entry
    int nb = 1;
    for (;; nb++) {
        double worst = 0;
        for (int bt = 0; bt < nb; bt++) {
            long long q = 0, leaf = 0, lv[kBfMaxLv + 1] = {};
            for (int m = bt; m <= L; m += nb)
                for (int t = 0; t < 2; t++) {
                    const size_t ii = (size_t)2 * m + t;
                    q += K;
                    leaf += item_leaf[ii];
                    for (int i = 1; i <= kBfMaxLv; i++) lv[i] += item_lvl[ii * (kBfMaxLv + 1) + i];
                }
            long long r0 = 0, r1 = 0;
            for (int i = 1; i <= kBfMaxLv; i++) (i & 1 ? r1 : r0) = std::max(i & 1 ? r1 : r0, lv[i]);
            worst = std::max(worst, 64.0 * (double)(q + leaf + r0 + r1));
        }
        if (worst <= target || nb > L) break;
    }
    b.nbatch = nb;
    b.batch_task.assign(nb + 1, 0);
    b.batch_sub.assign(nb + 1, 0);
    b.lv_off.assign((size_t)nb * (kBfMaxLv + 1) + 1, 0);
    b.f1_off.assign(nb + 1, 0);
    b.l1_off.assign(nb + 1, 0);
    b.fold_off.assign(nb + 1, 0);
    b.lv_max_n.assign((size_t)nb * kBfMaxLv, 0);
    b.batch_count.assign(nb, 0);
    for (int bt = 0; bt < nb; bt++) {
        long long leaf_cnt = 0, lvl_cnt[kBfMaxLv + 1] = {};
        int lvl_max_n[kBfMaxLv + 1] = {};
        std::vector<std::vector<int>> lvnodes(kBfMaxLv + 1);  // per level: node records
        std::vector<int> task_region;                          // per task: region of its output
        b.batch_task[bt] = (long long)b.res_task.size() / 8;
        const size_t task0 = b.res_task.size() / 8;
        int slot = 0;
        for (int m = bt; m <= L; m += nb, slot++) {
            for (int t = 0; t < 2; t++) {
                Item &it = c.items[(size_t)2 * m + t];
                const int d = it.depth;
                b.depth[(size_t)2 * m + t] = d;
                b.T_entries += it.T_entries;
                b.res_elems += it.res_elems;
                b.depth_hist[std::min(d, kBfMaxLv)]++;
                const long long qbase = (long long)(2 * slot + t) * K;
                // offsets of this item's vectors at every level it has
                std::vector<std::vector<long long>> voff(d + 1);
                std::vector<int> vreg(d + 1, RQ);
                for (int i = 1; i <= d; i++) {
                    const auto &lvn = it.lv[i - 1];
                    voff[i].resize(lvn.size());
                    long long *cnt = (i == d) ? &leaf_cnt : &lvl_cnt[i];
                    vreg[i] = (i == d) ? RLEAF : ((i & 1) ? RR1 : RR0);
                    for (size_t q = 0; q < lvn.size(); q++) {
                        voff[i][q] = *cnt;
                        *cnt += lvn[q].k;
                    }
                }
                // residual tasks
                const long long rbase = d == 0 ? qbase : (voff[d].empty() ? 0 : voff[d][0]);
                const int rreg = d == 0 ? RQ : RLEAF;
                for (size_t q = 0; q + 3 < it.seg.size(); q += 4) {
                    const int l0 = it.seg[q], l1 = it.seg[q + 1], rend = it.seg[q + 3];
                    const int cnt = l1 - l0;
                    if (cnt <= 0) continue;
                    const int ntask = (cnt + kBfTaskRings - 1) / kBfTaskRings;
                    for (int tk = 0; tk < ntask; tk++) {
                        const int c0 = l0 + (int)((long long)cnt * tk / ntask);
                        const int c1 = l0 + (int)((long long)cnt * (tk + 1) / ntask);
                        const int nl = c1 - c0;
                        int imin = rend;
                        for (int j = 0; j < nl; j++) imin = std::min(imin, it.lane[4 * (c0 + j) + 1]);
                        b.res_task.insert(b.res_task.end(),
                                          {t, imin, rend, nl, (int)(rbase + it.lane[4 * c0 + 3]), m, 0, 0});
                        task_region.push_back(rreg);
                        for (int j = 0; j < kBfTaskRings; j++) {
                            if (j < nl) {
                                const int *ln = &it.lane[4 * (c0 + j)];
                                b.res_lane.insert(b.res_lane.end(), {ln[0], ln[1]});
                                b.res_val.push_back(it.lval[2 * (c0 + j)]);
                                b.res_val.push_back(it.lval[2 * (c0 + j) + 1]);
                            } else {
                                b.res_lane.insert(b.res_lane.end(), {0, INT32_MAX});
                                b.res_val.push_back(0.0);
                                b.res_val.push_back(0.0);
                            }
                        }
                        b.n_res_lanes += nl;
                    }
                }
                // pair nodes of every level
                for (int lvl = d; lvl >= 1; lvl--) {
                    const int G = groups_at(it, lvl);
                    for (int pi = 0; pi < (1 << (lvl - 1)); pi++)
                        for (int g = 0; g < G; g++) {
                            const size_t q0 = (size_t)(2 * pi) * G + g, q1 = (size_t)(2 * pi + 1) * G + g;
                            const Node &c0 = it.lv[lvl - 1][q0];
                            const Node &c1 = it.lv[lvl - 1][q1];
                            const int nn = c0.n;  // both children share the columns C
                            if (nn == 0) continue;
                            long long out;
                            int oreg;
                            if (lvl == 1) {
                                out = qbase + it.colb[g];
                                oreg = RQ;
                            } else {
                                out = voff[lvl - 1][(size_t)pi * groups_at(it, lvl - 1) + 2 * g];
                                oreg = vreg[lvl - 1];
                            }
                            std::vector<int> &rec = lvnodes[lvl];
                            const long long T0 = (long long)b.T.size(), T1 = T0 + (long long)c0.T.size();
                            rec.insert(rec.end(), {(int)voff[lvl][q0], (int)voff[lvl][q1], c0.k, c1.k, c0.n - c0.k,
                                                   c1.n - c1.k, (int)out, (int)b.perm.size(), vreg[lvl] | (oreg << 2),
                                                   m, t, lvl, (int)(T0 & 0xffffffff), (int)(T0 >> 32),
                                                   (int)(T1 & 0xffffffff), (int)(T1 >> 32)});
                            for (const Node *ch : {&c0, &c1}) b.T.insert(b.T.end(), ch->T.begin(), ch->T.end());
                            // per child: skeleton positions (s order), then dense positions (d order)
                            for (const Node *ch : {&c0, &c1}) {
                                std::vector<int16_t> sk(ch->k), dn(nn - ch->k);
                                for (int q = 0; q < nn; q++) {
                                    const int cd = ch->code[q];
                                    if (cd >= 0)
                                        sk[cd] = (int16_t)q;
                                    else
                                        dn[-1 - cd] = (int16_t)q;
                                }
                                b.perm.insert(b.perm.end(), sk.begin(), sk.end());
                                b.perm.insert(b.perm.end(), dn.begin(), dn.end());
                            }
                            b.n_nodes++;
                            b.n_units += nn;
                            b.level_T[lvl] += (long long)(c0.T.size() + c1.T.size());
                            b.level_units[lvl] += nn;
                            b.level_nodes[lvl]++;
                            b.max_n = std::max(b.max_n, nn);
                            lvl_max_n[lvl] = std::max(lvl_max_n[lvl], nn);
                        }
                }
                std::vector<std::vector<Node>>().swap(it.lv);
                std::vector<int>().swap(it.lane);
                std::vector<double>().swap(it.lval);
                std::vector<int>().swap(it.seg);
            }
        }
        b.batch_count[bt] = slot;
        // batch-local region bases and absolute offsets
        long long r0 = 0, r1 = 0;
        for (int i = 1; i <= kBfMaxLv; i++) (i & 1 ? r1 : r0) = std::max(i & 1 ? r1 : r0, lvl_cnt[i]);
        const long long qsz = 2LL * K * slot;
        const long long base[4] = {0, qsz, qsz + leaf_cnt, qsz + leaf_cnt + r0};
        b.ws_entries = std::max(b.ws_entries, base[3] + r1);
        if (b.ws_entries > INT32_MAX || (long long)b.perm.size() > INT32_MAX)
            return fail(SHT_EUNSUPPORTED, "butterfly plan exceeds 32-bit record offsets");
        for (size_t q = 0; q < task_region.size(); q++) b.res_task[8 * (task0 + q) + 4] += (int)base[task_region[q]];
        // the same tasks in pieces of up to kBfPieceRings rings (one wave) for
        // the forward kernel, each starting at its own first row
        b.batch_sub[bt] = (long long)b.res_sub.size() / 8;
        for (size_t tk = task0; tk < b.res_task.size() / 8; tk++) {
            const int *h = &b.res_task[8 * tk];
            for (int q0 = 0; q0 < h[3]; q0 += kBfPieceRings) {
                const int nq = std::min(kBfPieceRings, h[3] - q0);
                int imin = h[2];
                for (int j = 0; j < nq; j++)
                    imin = std::min(imin, b.res_lane[2 * (tk * kBfTaskRings + q0 + j) + 1]);
                b.res_sub.insert(b.res_sub.end(),
                                 {h[0], imin, h[2], nq, h[4] + q0, h[5], (int)(tk * kBfTaskRings + q0), 0});
                b.res_exec += (long long)(h[2] - imin) * kBfPieceRings;
            }
        }
        // node records, deepest level first, with their launch ranges
        for (int lvl = kBfMaxLv; lvl >= 1; lvl--) {
            b.lv_off[(size_t)bt * (kBfMaxLv + 1) + kBfMaxLv - lvl] = (long long)b.node_i.size() / kBfNodeInts;
            b.lv_max_n[(size_t)bt * kBfMaxLv + kBfMaxLv - lvl] = lvl_max_n[lvl];
            std::vector<int> &rec = lvnodes[lvl];
            for (size_t q = 0; q < rec.size(); q += kBfNodeInts) {
                const int fl = rec[q + 8];
                rec[q + 0] += (int)base[fl & 3];
                rec[q + 1] += (int)base[fl & 3];
                rec[q + 6] += (int)base[(fl >> 2) & 3];
            }
            b.node_i.insert(b.node_i.end(), rec.begin(), rec.end());
            std::vector<int>().swap(rec);
            if (lvl != 1) continue;
            // level 1: pair the even and odd nodes of an order over the same
            // ring chunk (both parities share the chunk boundaries) when both
            // parities have levels; otherwise run them alone and fold later
            const long long l1a = b.lv_off[(size_t)bt * (kBfMaxLv + 1) + kBfMaxLv - 1];
            const long long l1b = (long long)b.node_i.size() / kBfNodeInts;
            b.f1_off[bt] = (long long)b.f1_unit.size() / 4;
            b.l1_off[bt] = (long long)b.l1_plain.size();
            b.fold_off[bt] = (long long)b.fold_slot.size();
            std::vector<std::vector<std::pair<int, int>>> per_m(slot);  // (k0 * 2 + t, node)
            for (long long nd = l1a; nd < l1b; nd++) {
                const int *ni = &b.node_i[(size_t)nd * kBfNodeInts];
                const int m = ni[9], t = ni[10], sl = (m - bt) / nb;
                const int k0 = ni[6] - (2 * sl + t) * K;
                per_m[sl].push_back({2 * k0 + t, (int)nd});
            }
            for (int sl = 0; sl < slot; sl++) {
                const int m = bt + sl * nb;
                auto &v = per_m[sl];
                std::sort(v.begin(), v.end());
                bool fuse = b.depth[(size_t)2 * m] >= 1 && b.depth[(size_t)2 * m + 1] >= 1 && v.size() % 2 == 0;
                for (size_t i = 0; fuse && i < v.size(); i += 2)
                    fuse = (v[i].first & 1) == 0 && v[i + 1].first == v[i].first + 1;
                if (fuse) {
                    for (size_t i = 0; i < v.size(); i += 2)
                        b.f1_unit.insert(b.f1_unit.end(), {v[i].second, v[i + 1].second, v[i].first / 2, sl});
                } else {
                    for (auto &x : v) b.l1_plain.push_back(x.second);
                    b.fold_slot.push_back(sl);
                }
            }
        }
        b.lv_off[(size_t)bt * (kBfMaxLv + 1) + kBfMaxLv] = (long long)b.node_i.size() / kBfNodeInts;
    }
    b.batch_task[nb] = (long long)b.res_task.size() / 8;
    b.f1_off[nb] = (long long)b.f1_unit.size() / 4;
    b.l1_off[nb] = (long long)b.l1_plain.size();
    b.fold_off[nb] = (long long)b.fold_slot.size();
    b.batch_sub[nb] = (long long)b.res_sub.size() / 8;
    if ((long long)b.res_lane.size() / 2 > INT32_MAX)
        return fail(SHT_EUNSUPPORTED, "butterfly plan exceeds 32-bit lane record offsets");
    // every level launch keeps its workgroup's vectors in the default 64 KiB
    // of dynamic LDS at 8 maps in FP64: the fused level 1 holds four vectors
    // of n entries (128 B each), the other levels two
    long long n1 = 0, nl = 0;
    for (int bt = 0; bt < nb; bt++)
        for (int q = 0; q < kBfMaxLv; q++) {
            const long long n = b.lv_max_n[(size_t)bt * kBfMaxLv + q];
            if (q == kBfMaxLv - 1) n1 = std::max(n1, n);
            else nl = std::max(nl, n);
        }
    if (512 * n1 > 65536 || 256 * nl > 65536)
        return fail(SHT_EUNSUPPORTED, "butterfly column sets too wide for the level kernels' LDS (use a smaller chunk)");
    b.n_tasks = (long long)b.res_task.size() / 8;
    b.built = 1;
    b.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return SHT_OK;
}

// ---------------------------------------------------------------------
// Host evaluation of q^t_m = Lambda^T x from the flattened records (test
// support: checks the factorization without a GPU).  x: n_t doubles (real
// coefficients of the rows), y: K doubles.
// ---------------------------------------------------------------------
static long long node_T_off(const int *ni, int ch) {
    return (long long)(unsigned)ni[12 + 2 * ch] | ((long long)ni[13 + 2 * ch] << 32);
}

int butterfly_apply_host(const sht_plan_s *p, int m, int t, const double *x, double *y) {
    const BflyPlan &b = p->bf;
    const int K = b.K;
    const int bt = m % b.nbatch, slot = m / b.nbatch;
    std::vector<double> ws((size_t)b.ws_entries, 0.0);
    const double *cf = p->coef_hi.data() + 4 * p->coef_off[m];
    for (long long tk = b.batch_task[bt]; tk < b.batch_task[bt + 1]; tk++) {
        const int *h = &b.res_task[(size_t)8 * tk];
        if (h[0] != t || h[5] != m) continue;
        for (int j = 0; j < h[3]; j++) {
            const size_t li = (size_t)tk * kBfTaskRings + j;
            const int k = b.res_lane[2 * li], i0 = b.res_lane[2 * li + 1];
            double P0 = b.res_val[2 * li], P1 = b.res_val[2 * li + 1], acc = 0.0;
            const double z2 = p->z2_hi[k];
            for (int i = i0; i < h[2]; i++) {
                acc += P0 * x[i];
                const double *e = cf + 4 * (t + 2 * i + 2);
                double P2 = (z2 * e[0] + e[1]) * P1 + e[2] * P0;
                P0 = P1;
                P1 = P2;
            }
            ws[(size_t)h[4] + j] = acc;
        }
    }
    const long long *lo = b.lv_off.data() + (size_t)bt * (kBfMaxLv + 1);
    for (int q = 0; q < kBfMaxLv; q++) {
        for (long long node = lo[q]; node < lo[q + 1]; node++) {
            const int *ni = &b.node_i[(size_t)node * kBfNodeInts];
            if (ni[9] != m || ni[10] != t) continue;
            const int n = ni[2] + ni[4];
            std::vector<double> u(n, 0.0);
            for (int ch = 0; ch < 2; ch++) {
                const int16_t *pm = b.perm.data() + ni[7] + (size_t)ch * n;
                const int kk = ni[2 + ch], nd = ni[4 + ch];
                const double *v = ws.data() + ni[ch];
                const double *Tp = b.T.data() + node_T_off(ni, ch);
                for (int s2 = 0; s2 < kk; s2++) u[pm[s2]] += v[s2];
                for (int d = 0; d < nd; d++) {
                    double acc = 0.0;
                    for (int s2 = 0; s2 < kk; s2++) acc += Tp[(size_t)s2 * nd + d] * v[s2];
                    u[pm[kk + d]] += acc;
                }
            }
            for (int c2 = 0; c2 < n; c2++) ws[(size_t)ni[6] + c2] = u[c2];
        }
    }
    const size_t q = (size_t)(2 * slot + t) * K;
    for (int k = 0; k < K; k++) y[k] = ws[q + k];
    return SHT_OK;
}

}  // namespace sht
