// Host precompute of the butterfly-compressed Legendre operator (Sec. 4 of
// the Wavemoth paper), and its flattening into the records the GPU kernel
// walks.
//
// For each order m and parity t the matrix Lambda (rows: l = m + t + 2i,
// i = 0..n-1; columns: the north rings z_k) is factored as in Sec. 4.2,
// Eq. 15: Lambda = R S_d P_{d-1} ... P_1 S_1.  Level 1 splits the rows in
// two and takes the interpolative decomposition (Sec. 4.1, Eq. 16) of every
// (row half, column block of about `chunk` rings); level i > 1 joins the
// skeleton columns that two neighbouring level-(i-1) column groups kept in
// the same parent row block, splits the rows again and takes the ID of each
// half (Eq. 18).  After d levels the residual R consists of, per leaf (row
// block, column group), the Legendre values at the leaf's rows and its
// skeleton rings; the kernel regenerates those with the recurrence from two
// stored values per column (Sec. 4.4), so only the interpolation matrices
// (their dense, non-identity part, App. A.1) are streamed from memory.
//
// The depth d of each (m, t) minimises rho * (stored interpolation entries)
// + (residual recurrence elements), the paper's CPU/memory trade-off of
// Sec. 4.4 with rho set for MI355X instead of a CPU.
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
            for (int q = j + 1; q < c; q++) {
                double *cq = A + (size_t)q * r;
                double w = cq[j];
                for (int i = j + 1; i < r; i++) w += v[i] * cq[i];
                w *= tau;
                cq[j] -= w;
                for (int i = j + 1; i < r; i++) cq[i] -= w * v[i];
            }
        }
        // downdate the remaining column norms (recompute on cancellation)
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
    // T = R11^{-1} R12
    const int nd = c - k;
    T.assign((size_t)k * nd, 0.0);
    for (int d = 0; d < nd; d++) {
        const double *cq = A + (size_t)(k + d) * r;
        for (int s = k - 1; s >= 0; s--) {
            double acc = cq[s];
            for (int s2 = s + 1; s2 < k; s2++) acc -= A[(size_t)s2 * r + s] * T[(size_t)s2 * nd + d];
            T[(size_t)s * nd + d] = acc / A[(size_t)s * r + s];
        }
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
        for (int k = 0; k < K; k++) lane(k, 0, n, k);
    } else {
        const int d = it.depth, G = groups_at(it, d);
        int off = 0;
        for (int rho = 0; rho < (1 << d); rho++) {
            int r0, r1;
            row_bounds(n, d, rho, &r0, &r1);
            for (int g = 0; g < G; g++) {
                const Node &nd = it.lv[d - 1][(size_t)rho * G + g];
                for (int s = 0; s < nd.k; s++) lane(nd.skel[s], r0, r1, off + s);
                off += nd.k;
            }
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
    c.eps_id = p->eps / std::max(1.0, p->opts.id_safety);
    c.rho = p->opts.rho > 0 ? p->opts.rho : 2.5;
    c.chunk = p->opts.chunk > 0 ? p->opts.chunk : 64;
    c.max_levels = p->opts.max_levels;
    parallel_for((long)c.items.size(), p->opts.nthreads, item_worker, &c);

    BflyPlan &b = p->bf;
    b = BflyPlan();
    b.K = K;
    {
        size_t nT = 0, nl = 0;
        for (auto &it : c.items) {
            nT += (size_t)it.T_entries;
            nl += it.lane.size() / 4;
        }
        b.T.reserve(nT);
        b.res_rec.reserve(4 * nl);
        b.res_val.reserve(2 * nl);
    }
    b.depth.assign((size_t)(L + 1) * 2, 0);
    b.res_off.assign(L + 2, 0);
    b.unit_off.assign((size_t)(L + 1) * (kBfMaxLv + 1), 0);
    // per-parity vector region size: the largest level vector of any item
    long long vmax = 1;
    for (auto &it : c.items)
        for (auto &lvn : it.lv) {
            long long s = 0;
            for (auto &nd : lvn) s += nd.k;
            vmax = std::max(vmax, s);
        }
    b.vmax = vmax;
    b.slot_entries = 2LL * K + 4 * vmax;
    auto region = [&](int t, int i) -> long long { return 2LL * K + (2LL * t + (i & 1)) * vmax; };

    std::vector<double> work(L + 1, 0.0);
    for (int m = 0; m <= L; m++) {
        b.res_off[m] = (long long)b.res_rec.size() / 4;
        int dm = 0;
        for (int t = 0; t < 2; t++) {
            Item &it = c.items[(size_t)2 * m + t];
            b.depth[(size_t)2 * m + t] = it.depth;
            b.T_entries += it.T_entries;
            b.res_elems += it.res_elems;
            b.depth_hist[std::min(it.depth, kBfMaxLv)]++;
            work[m] += c.rho * (double)it.T_entries + (double)it.res_elems;
            dm = std::max(dm, it.depth);
        }
        // residual lanes: leaves of the deepest level kept (or every ring)
        for (int t = 0; t < 2; t++) {
            Item &it = c.items[(size_t)2 * m + t];
            const long long base = it.depth == 0 ? (long long)t * K : region(t, it.depth);
            const size_t nl = it.lane.size() / 4;
            for (size_t q = 0; q < nl; q++) {
                const int *ln = &it.lane[4 * q];
                b.res_rec.insert(b.res_rec.end(), {ln[0], ln[1], ln[2], (int)((base + ln[3]) * 2 + t)});
                b.res_val.push_back(it.lval[2 * q]);
                b.res_val.push_back(it.lval[2 * q + 1]);
            }
            std::vector<int>().swap(it.lane);
            std::vector<double>().swap(it.lval);
        }
        // level records, deepest first; level i of parity t reads region (t, i)
        // and writes region (t, i-1) (level 1 writes the q^t rows)
        for (int lvl = kBfMaxLv; lvl >= 1; lvl--) {
            b.unit_off[(size_t)m * (kBfMaxLv + 1) + kBfMaxLv - lvl] = (long long)b.unit_node.size();
            if (lvl > dm) continue;
            for (int t = 0; t < 2; t++) {
                Item &it = c.items[(size_t)2 * m + t];
                if (lvl > it.depth) continue;
                const int G = groups_at(it, lvl);
                // input offsets of level lvl vectors (node order rho-major)
                std::vector<long long> vin((size_t)(1 << lvl) * G);
                long long off = region(t, lvl);
                for (size_t q = 0; q < vin.size(); q++) {
                    vin[q] = off;
                    off += it.lv[lvl - 1][q].k;
                }
                std::vector<long long> vout;
                if (lvl > 1) {
                    const int Gp = groups_at(it, lvl - 1);
                    vout.resize((size_t)(1 << (lvl - 1)) * Gp);
                    long long o2 = region(t, lvl - 1);
                    for (size_t q = 0; q < vout.size(); q++) {
                        vout[q] = o2;
                        o2 += it.lv[lvl - 2][q].k;
                    }
                }
                for (int pi = 0; pi < (1 << (lvl - 1)); pi++)
                    for (int g = 0; g < G; g++) {
                        const Node &c0 = it.lv[lvl - 1][(size_t)(2 * pi) * G + g];
                        const Node &c1 = it.lv[lvl - 1][(size_t)(2 * pi + 1) * G + g];
                        const int nn = c0.n;  // both children share the columns C
                        if (nn == 0) continue;
                        const int node = (int)(b.node_i.size() / kBfNodeInts);
                        long long out = lvl > 1 ? vout[(size_t)pi * groups_at(it, lvl - 1) + 2 * g]
                                                : (long long)t * K + it.colb[g];
                        const long long ubase = (long long)b.unit_node.size();
                        b.node_i.insert(b.node_i.end(),
                                        {(int)vin[(size_t)(2 * pi) * G + g], (int)vin[(size_t)(2 * pi + 1) * G + g],
                                         c0.k, c1.k, c0.n - c0.k, c1.n - c1.k, (int)out, (int)ubase});
                        b.node_T.push_back((long long)b.T.size());
                        b.T.insert(b.T.end(), c0.T.begin(), c0.T.end());
                        b.node_T.push_back((long long)b.T.size());
                        b.T.insert(b.T.end(), c1.T.begin(), c1.T.end());
                        for (int q = 0; q < nn; q++) {
                            b.unit_node.push_back(node);
                            b.code.push_back((c0.code[q] & 0xffff) | (int)((unsigned)(c1.code[q] & 0xffff) << 16));
                        }
                        b.n_nodes++;
                    }
            }
        }
        b.unit_off[(size_t)m * (kBfMaxLv + 1) + kBfMaxLv] = (long long)b.unit_node.size();
        // free the item's trees
        for (int t = 0; t < 2; t++) {
            Item &it = c.items[(size_t)2 * m + t];
            std::vector<std::vector<Node>>().swap(it.lv);
        }
    }
    b.res_off[L + 1] = (long long)b.res_rec.size() / 4;
    b.order.resize(L + 1);
    std::iota(b.order.begin(), b.order.end(), 0);
    std::stable_sort(b.order.begin(), b.order.end(), [&](int x, int y) { return work[x] > work[y]; });
    if (b.slot_entries > INT32_MAX / 2 || (long long)b.unit_node.size() > INT32_MAX)
        return fail(SHT_EUNSUPPORTED, "butterfly plan exceeds 32-bit record offsets");
    b.built = 1;
    b.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return SHT_OK;
}

// ---------------------------------------------------------------------
// Host evaluation of q^t_m = Lambda^T x from the flattened records (test
// support: checks the factorization without a GPU).  x: n_t doubles (real
// coefficients of the rows), y: K doubles.
// ---------------------------------------------------------------------
int butterfly_apply_host(const sht_plan_s *p, int m, int t, const double *x, double *y) {
    const BflyPlan &b = p->bf;
    const int K = b.K;
    std::vector<double> slot((size_t)b.slot_entries, 0.0);
    const double *cf = p->coef_hi.data() + 4 * p->coef_off[m];
    for (long long r = b.res_off[m]; r < b.res_off[m + 1]; r++) {
        const int *rec = &b.res_rec[(size_t)4 * r];
        if ((rec[3] & 1) != t) continue;
        const int k = rec[0], i0 = rec[1], i1 = rec[2];
        const long long out = rec[3] >> 1;
        double P0 = b.res_val[2 * r], P1 = b.res_val[2 * r + 1], acc = 0.0;
        const double z2 = p->z2_hi[k];
        for (int i = i0; i < i1; i++) {
            acc += P0 * x[i];
            const double *e = cf + 4 * (t + 2 * i + 2);
            double P2 = (z2 * e[0] + e[1]) * P1 + e[2] * P0;
            P0 = P1;
            P1 = P2;
        }
        slot[out] = acc;
    }
    for (int q = 0; q < kBfMaxLv; q++) {
        for (long long u = b.unit_off[(size_t)m * (kBfMaxLv + 1) + q];
             u < b.unit_off[(size_t)m * (kBfMaxLv + 1) + q + 1]; u++) {
            const int node = b.unit_node[u];
            const int *ni = &b.node_i[(size_t)node * kBfNodeInts];
            // parity of the node: its output lies in the q^t rows or a parity region
            const long long out = ni[6];
            const int tn = out < 2LL * K ? (int)(out / K) : (int)((out - 2LL * K) / (2 * b.vmax));
            if (tn != t) continue;
            const int c = (int)(u - ni[7]);
            const int code = b.code[u];
            double acc = 0.0;
            for (int ch = 0; ch < 2; ch++) {
                const int cd = (int16_t)((ch == 0 ? code : (code >> 16)) & 0xffff);
                const long long vin = ni[ch];
                if (cd >= 0) {
                    acc += slot[vin + cd];
                } else {
                    const int d = -1 - cd, kk = ni[2 + ch], nd = ni[4 + ch];
                    const double *Tp = b.T.data() + b.node_T[(size_t)2 * node + ch];
                    for (int s = 0; s < kk; s++) acc += Tp[(size_t)s * nd + d] * slot[vin + s];
                }
            }
            slot[out + c] = acc;
        }
    }
    for (int k = 0; k < K; k++) y[k] = slot[(size_t)t * K + k];
    return SHT_OK;
}

}  // namespace sht
