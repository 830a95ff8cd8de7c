// Butterfly-compressed Legendre phase for gfx950 (Sec. 3.2 and App. A.1 of
// the Wavemoth paper): q^t_m = Lambda^T a^t applied as
//   a^T Lambda = (a^T R) S_d P_{d-1} ... P_1 S_1,
// followed by the even/odd fold of Sec. 2.4 (Eqs. 13-14).
//
// The paper walks each order's tree depth first to stay in a CPU's caches.
// Here every level is one launch over all orders at once (breadth first),
// which gives the GPU tens of thousands of independent waves to stream the
// interpolation matrices with; vectors between levels live in a device
// workspace (read and written once per level):
//  1. k_bf_residual: one wave per residual piece (up to kBfPieceRings skeleton
//     rings of one row block, four per lane) regenerates the Legendre values with the
//     two-step recurrence (App. A.2, Eq. A2) over the block's rows from two
//     stored values per ring and accumulates v = sum_l a_lm P~_l^m(z) for
//     every map; the a_lm rows and coefficients are staged through LDS;
//  2. k_bf_level, deepest level first down to level 2: one workgroup (a wave
//     per child) per pair node (two sibling row blocks sharing the column set
//     C) computes u = A~_0^T v_0 + A~_1^T v_1: identity rows copy v, the
//     dense part T^T V runs on the matrix cores;
//  3. level 1 yields q^even and q^odd per north ring: k_bf_level1_fold runs
//     the two level-1 nodes of one order and ring range together and writes
//     q rows k and 4 nside - k from q^even +- q^odd (Eqs. 13-14); orders
//     whose parities split differently run k_bf_level_list, then k_bf_fold.
//
// The adjoint runs the same factorization backwards in butterfly_adjoint.hip.
#include <cstring>

#include "butterfly_common.h"

namespace sht {


// One ID block (child ch of a pair node) on one wave: child ch's share of
//   u = A~_0^T v_0 + A~_1^T v_1
// over the columns C the two sibling row blocks share.  Its column
// permutation places every column of C exactly once, as a skeleton column
// (u[perm s] = v[s]) or a dense one (u[perm (k + d)] = sum_s T[s][d] v[s]),
// so the wave writes each entry of its own LDS buffer uc once, with plain
// stores, and the two buffers are summed afterwards.  The dense part T^T V
// (nd x k times k x NC) runs on the matrix cores, up to 64 dense rows (four
// 16-row tiles sharing each V operand) by kBfKSteps * 4 rows of T per batch
// of loads.  Loads take clamped (in-block) addresses and rows s past k are
// masked by multiplying V with 0, so a batch issues all its loads without
// branches; dense rows past nd and columns past NC only reach outputs that
// are not stored.
constexpr int kBfKSteps = 4;    // K-steps (4 rows of T each) per batch of loads
constexpr int kBfIdUnroll = 4;  // identity entries per lane in flight

// NT 16-row tiles of dense rows gw .. gw + 16 NT - 1 of one ID block:
// uc[perm (k + d)] = sum_s T[s][d] v[s] (32-bit element offsets from
// wave-uniform bases; the tile count is a template parameter so that the
// products run back to back, without branches between them).
template <int NT, int NB, typename S>
__device__ __forceinline__ void dense_tiles(const S *__restrict__ v, int ES, const S *__restrict__ Tb,
                                            const int16_t *__restrict__ pm, int kk, int nd, int gw, int lane,
                                            S *uc) {
    constexpr int NC = 2 * NB;
    constexpr int KS = kBfKSteps;
    typedef typename Acc<S>::type acc_t;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int ic = min(i16, NC - 1);
    acc_t acc[NT];
#pragma unroll
    for (int tt = 0; tt < NT; tt++) acc[tt] = acc_t{0, 0, 0, 0};
    for (int s0 = 0; s0 < kk; s0 += 4 * KS) {
        S av[KS][NT], bv[KS];
#pragma unroll
        for (int j = 0; j < KS; j++) {
            const int s = s0 + 4 * j + k4, sc = min(s, kk - 1);
            bv[j] = ld32(v, sc * ES + ic) * (S)(s < kk);
#pragma unroll
            for (int tt = 0; tt < NT; tt++) av[j][tt] = ld32(Tb, sc * nd + min(gw + 16 * tt + i16, nd - 1));
        }
#pragma unroll
        for (int j = 0; j < KS; j++)
#pragma unroll
            for (int tt = 0; tt < NT; tt++) acc[tt] = mfma_16x16x4(av[j][tt], bv[j], acc[tt]);
    }
    // the output rows' positions in C, all loads issued before the first
    // store (the empty asm keeps the compiler from moving each load into
    // its store's branch, which would wait on them one by one)
    int pr[NT][4];
#pragma unroll
    for (int tt = 0; tt < NT; tt++)
#pragma unroll
        for (int r = 0; r < 4; r++) pr[tt][r] = pm[kk + min(gw + 16 * tt + acc_row<S>(k4, r), nd - 1)];
    asm volatile("" ::: "memory");
#pragma unroll
    for (int tt = 0; tt < NT; tt++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int dd = gw + 16 * tt + acc_row<S>(k4, r);
            if (dd < nd && i16 < NC) uc[pr[tt][r] * NC + i16] = acc[tt][r];
        }
}

template <int NB, typename S, bool ONE>
__device__ __forceinline__ void id_block(const BfArgs<S> &a, int node, int ch, int half, int lane, S *uc, int col) {
    constexpr int NC = 2 * NB;
    constexpr int TPW = 4 / kBfHalves;  // tiles per wave
    constexpr int KS = kBfKSteps;
    typedef typename Acc<S>::type acc_t;
    const int *ni = a.node_i + (size_t)node * kBfNodeInts;
    const int n = ni[2] + ni[4];
    const int kk = ni[2 + ch], nd = ni[4 + ch];
    const int ES = ONE ? NC : a.ES;  // one group per pass: the stride is a constant
    const S *__restrict__ v = a.ws + (size_t)ni[ch] * ES + col;
    const int16_t *__restrict__ pm = a.perm + ni[7] + (size_t)ch * n;
    const long long toff = (long long)(unsigned)ni[12 + 2 * ch] | ((long long)ni[13 + 2 * ch] << 32);
    const S *__restrict__ Tb = a.T + toff;
    // identity rows (lanes past the end repeat the last entry's store)
    const int ne = kk * NC;
    for (int e0 = 64 * half; e0 < ne; e0 += 64 * kBfHalves * kBfIdUnroll) {
        S x[kBfIdUnroll];
        int px[kBfIdUnroll];
#pragma unroll
        for (int j = 0; j < kBfIdUnroll; j++) {
            const int ec = min(e0 + lane + 64 * kBfHalves * j, ne - 1);
            x[j] = ld32(v, (ec / NC) * ES + ec % NC);
            px[j] = pm[ec / NC];
        }
#pragma unroll
        for (int j = 0; j < kBfIdUnroll; j++) {
            const int ec = min(e0 + lane + 64 * kBfHalves * j, ne - 1);
            uc[px[j] * NC + ec % NC] = x[j];
        }
    }
    // dense rows, in groups of 64
    for (int g0 = 0; g0 < nd; g0 += 64) {
        const int ntile = min(TPW, min(4, (nd - g0 + 15) >> 4) - half * TPW);  // tiles of this wave
        const int gw = g0 + 16 * TPW * half;
        switch (ntile) {
            case 1: dense_tiles<1, NB, S>(v, ES, Tb, pm, kk, nd, gw, lane, uc); break;
            case 2: dense_tiles<2, NB, S>(v, ES, Tb, pm, kk, nd, gw, lane, uc); break;
            case 3: dense_tiles<3, NB, S>(v, ES, Tb, pm, kk, nd, gw, lane, uc); break;
            case 4: dense_tiles<4, NB, S>(v, ES, Tb, pm, kk, nd, gw, lane, uc); break;
            default: break;
        }
    }
}

// acc[c] += x_c * p for c < N, where x_c is the value that lane c of the
// lane's 16-lane row holds in rv: each FP64 FMA reads rv through the DPP
// broadcast (row_newbcast), so the per-row operands need neither one LDS
// broadcast read per value nor a register each.  One asm block per call:
// its leading s_nop gives the two wait states that a DPP read needs after a
// vector-ALU write of rv, and nothing can be scheduled inside it.
#define SHT_FMAC_BC(c, o) "v_fmac_f64_dpp %" #o ", %[rv], %[p] row_newbcast:" #c " row_mask:0xf bank_mask:0xf\n"
template <int N>
__device__ __forceinline__ void fmac_row_bcast(double *acc, double rv, double p);
template <>
__device__ __forceinline__ void fmac_row_bcast<2>(double *acc, double rv, double p) {
    asm("s_nop 1\n" SHT_FMAC_BC(0, 0) SHT_FMAC_BC(1, 1) : "+v"(acc[0]), "+v"(acc[1]) : [rv] "v"(rv), [p] "v"(p));
}
template <>
__device__ __forceinline__ void fmac_row_bcast<4>(double *acc, double rv, double p) {
    asm("s_nop 1\n" SHT_FMAC_BC(0, 0) SHT_FMAC_BC(1, 1) SHT_FMAC_BC(2, 2) SHT_FMAC_BC(3, 3)
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])
        : [rv] "v"(rv), [p] "v"(p));
}
template <>
__device__ __forceinline__ void fmac_row_bcast<8>(double *acc, double rv, double p) {
    asm("s_nop 1\n" SHT_FMAC_BC(0, 0) SHT_FMAC_BC(1, 1) SHT_FMAC_BC(2, 2) SHT_FMAC_BC(3, 3) SHT_FMAC_BC(4, 4)
            SHT_FMAC_BC(5, 5) SHT_FMAC_BC(6, 6) SHT_FMAC_BC(7, 7)
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]), "+v"(acc[6]),
          "+v"(acc[7])
        : [rv] "v"(rv), [p] "v"(p));
}
template <>
__device__ __forceinline__ void fmac_row_bcast<16>(double *acc, double rv, double p) {
    fmac_row_bcast<8>(acc, rv, p);
    asm("s_nop 1\n" SHT_FMAC_BC(8, 0) SHT_FMAC_BC(9, 1) SHT_FMAC_BC(10, 2) SHT_FMAC_BC(11, 3) SHT_FMAC_BC(12, 4)
            SHT_FMAC_BC(13, 5) SHT_FMAC_BC(14, 6) SHT_FMAC_BC(15, 7)
        : "+v"(acc[8]), "+v"(acc[9]), "+v"(acc[10]), "+v"(acc[11]), "+v"(acc[12]), "+v"(acc[13]), "+v"(acc[14]),
          "+v"(acc[15])
        : [rv] "v"(rv), [p] "v"(p));
}
#undef SHT_FMAC_BC

// The value of lane K of each 16-lane row, in every lane of that row.
template <int K>
__device__ __forceinline__ double row_bcast(double x) {
    return __builtin_amdgcn_mov_dpp(x, 0x150 + K, 0xF, 0xF, false);
}

// One residual piece on one wave: R rings per lane (lane j: rings j + 64 r,
// lane records from lbase), rows [imin, iend) of one parity, outputs at
// entries outb + ring.  The a_lm rows and recurrence coefficients of each
// aligned chunk of kChunk rows are fetched one chunk ahead with coalesced
// vector loads and staged in the wave's own LDS slot (stg: two chunks) as
// rows of 16 (NC <= 13) or 32 values: a_lm components, then B, AB and G.
// Lane k of every 16-lane row reads value k of a row, and the products take
// the values from there by DPP broadcasts; LDS operations of one wave
// complete in order, so no barrier is needed.
template <int NB>
constexpr int bf_res_row_doubles() {
    return 2 * NB + 3 <= 16 ? 16 : 32;
}
template <int NB>
constexpr int bf_res_stage_doubles() {
    return 2 * kChunk * bf_res_row_doubles<NB>();
}

template <int NB, int R, typename S>
__device__ __forceinline__ void residual_task(const BfArgs<S> &a, S *__restrict__ slot, long long lbase, int lane,
                                              int t, int imin, int iend, int nl, int outb,
                                              const double *__restrict__ ap, const double *__restrict__ cfs,
                                              int astride, double *stg, int col0) {
    constexpr int NC = 2 * NB;
    constexpr int CW = bf_res_row_doubles<NB>();  // staged values per row
    constexpr int CS = kChunk * CW;                // doubles per staged chunk
    constexpr int E = CS / 64;                     // staged doubles per lane
    constexpr int CO = NC < 16 ? NC : 0;           // lane of B within its 16-lane group
    int i0[R];
    double z2[R], v0[R], v1[R], P0[R], P1[R], acc[R][NC];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const size_t li = (size_t)lbase + r * 64 + lane;
        const int2 ln = a.res_lane[li];
        const double2 sv = a.res_val[li];
        i0[r] = ln.y;
        z2[r] = a.z2[ln.x];
        v0[r] = sv.x;
        v1[r] = sv.y;
        P0[r] = P1[r] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; c++) acc[r][c] = 0.0;
    }
    // Chunk loads without branches: every lane loads from a row clamped into
    // [imin, iend) and keeps zero where the row or the component lies outside,
    // so that a chunk's whole update is one basic block the compiler cannot
    // reorder around branches.
    double pre[E];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int e = 0; e < E; e++) {
            const int idx = lane + 64 * e, ir = c0 + idx / CW, comp = idx % CW;
            const int i = min(ir, iend - 1);
            const double *p = comp < NC ? ap + (size_t)i * astride + comp
                                        : cfs + 4 * (t + 2 * i + 2) + min(comp - NC, 2);
            const double v = *p;
            pre[e] = (ir < iend && comp < NC + 3) ? v : 0.0;
        }
    };
    auto stage = [&](int sl) {
#pragma unroll
        for (int e = 0; e < E; e++) stg[sl * CS + lane + 64 * e] = pre[e];
    };
    auto step_v = [&](double rv, double rc) {
        const double eb = row_bcast<CO>(rc), eab = row_bcast<CO + 1>(rc), eg = row_bcast<CO + 2>(rc);
#pragma unroll
        for (int r = 0; r < R; r++) {
            fmac_row_bcast<NC>(acc[r], rv, P0[r]);
            const double P2 = __builtin_fma(__builtin_fma(z2[r], eb, eab), P1[r], eg * P0[r]);
            P0[r] = P1[r];
            P1[r] = P2;
        }
    };
    auto step = [&](const double *row) {
        const double rv = row[lane & 15];
        step_v(rv, CW == 16 ? rv : row[16 + (lane & 15)]);
    };
    // a piece without rows (a parity with no l <= L) writes zeros and loads
    // nothing: its clamped row iend - 1 would lie outside the order's rows
    if (imin < iend) {
        int c0 = imin & ~(kChunk - 1), sl = 0;
        fetch(c0);
        stage(0);
        fetch(c0 + kChunk);
        // The rings that start at imin; a first chunk that begins before imin
        // runs row by row, every later chunk as eight unrolled steps (rows past
        // iend are staged as zeros, which leave the sums unchanged).
#pragma unroll
        for (int r = 0; r < R; r++)
            if (i0[r] == imin) {
                P0[r] = v0[r];
                P1[r] = v1[r];
            }
        if (c0 != imin) {
            const int ce = min(iend, c0 + kChunk);
            for (int i = imin; i < ce; i++) step(stg + (i - c0) * CW);
            stage(1);
            fetch(c0 + 2 * kChunk);
            c0 += kChunk;
            sl = 1;
        }
        for (; c0 < iend; c0 += kChunk, sl ^= 1) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                const bool st = i0[r] == c0;
                P0[r] = st ? v0[r] : P0[r];
                P1[r] = st ? v1[r] : P1[r];
            }
            // the chunk's rows are read at once (one or two values per lane
            // and row), so that their LDS latency is paid once per chunk
            const double *cur = stg + sl * CS + (lane & 15);
            double rv[kChunk], rc[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; u++) {
                rv[u] = cur[u * CW];
                rc[u] = CW == 16 ? rv[u] : cur[u * CW + 16];
            }
#pragma unroll
            for (int u = 0; u < kChunk; u++) step_v(rv[u], rc[u]);
            stage(sl ^ 1);
            fetch(c0 + 2 * kChunk);
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int j = r * 64 + lane;
        if (j < nl) {
            S *dst = slot + ((size_t)outb + j) * a.ES + col0;
#pragma unroll
            for (int c = 0; c < NC; c++) dst[c] = (S)acc[r][c];
        }
    }
}

// One wave per residual piece (up to kBfPieceRings skeleton rings of one
// task): short waves keep the register count, and with it the occupancy, low.
template <int NB, typename S>
__device__ __forceinline__ void residual_piece(const BfArgs<S> &a, long long tk, int lane, double *stg, int col0) {
    const int4 h = a.res_sub[2 * tk], h2 = a.res_sub[2 * tk + 1];
    const int t = __builtin_amdgcn_readfirstlane(h.x), imin = __builtin_amdgcn_readfirstlane(h.y);
    const int iend = __builtin_amdgcn_readfirstlane(h.z), nl = __builtin_amdgcn_readfirstlane(h.w);
    const int outb = __builtin_amdgcn_readfirstlane(h2.x), m = __builtin_amdgcn_readfirstlane(h2.y);
    const long long lbase = (unsigned)__builtin_amdgcn_readfirstlane(h2.z);
    const size_t aoff = (size_t)m * (2 * a.L + 3 - m) / 2;
    const double *ap = reinterpret_cast<const double *>(a.alm + (aoff + t) * a.nmaps + a.map0);
    const double *cfs = a.coef + 4 * a.coef_off[m];
    const int astride = 4 * a.nmaps;  // doubles between rows i and i+1
    residual_task<NB, kBfPieceRings / 64>(a, a.ws, lbase, lane, t, imin, iend, nl, outb, ap, cfs, astride, stg,
                                          col0);
}

template <int NB, typename S>
__global__ __launch_bounds__(kBfThreads) void k_bf_residual(BfArgs<S> a, long long t0, long long t1, int col0) {
    __shared__ double stg_all[kBfThreads / 64][bf_res_stage_doubles<NB>()];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long tk = t0 + (long long)blockIdx.x * (kBfThreads / 64) + w;
    if (tk >= t1) return;
    residual_piece<NB, S>(a, tk, threadIdx.x & 63, stg_all[w], col0);
}

// One workgroup of 2 kBfHalves waves per pair node (wave w: child w % 2,
// half w / 2): per group of NB maps, each child writes its share of u into
// its own LDS copy, and the two copies are summed into the next level's
// vector with one coalesced store.

template <int NB, typename S, bool ONE>
__device__ __forceinline__ void level_node_g(const BfArgs<S> &a, int node) {
    constexpr int NC = 2 * NB;
    extern __shared__ char lds_raw[];
    S *u0 = reinterpret_cast<S *>(lds_raw);
    const int *ni = a.node_i + (size_t)node * kBfNodeInts;
    const int n = ni[2] + ni[4];
    S *u1 = u0 + (size_t)n * NC;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ES = ONE ? NC : a.ES, G = ONE ? 1 : a.G;
    S *__restrict__ out = a.ws + (size_t)ni[6] * ES;
    for (int g = 0; g < G; g++) {
        if (g) __syncthreads();  // the previous group's sums have been read out of LDS
        id_block<NB, S, ONE>(a, node, w & 1, w >> 1, threadIdx.x & 63, (w & 1) ? u1 : u0, g * NC);
        __syncthreads();
        if (ONE) {
            for (int e = threadIdx.x; e < n * NC; e += kBfLevelThreads) out[e] = u0[e] + u1[e];
        } else {
            for (int e = threadIdx.x; e < n * NC; e += kBfLevelThreads)
                out[(size_t)(e / NC) * ES + g * NC + e % NC] = u0[e] + u1[e];
        }
    }
}


// ONE: the pass has a single group of maps (separate instantiations, so the
// common case keeps its constant strides and its register count).
template <int NB, typename S, bool ONE>
__global__ __launch_bounds__(kBfLevelThreads) void k_bf_level(BfArgs<S> a, long long n0) {
    level_node_g<NB, S, ONE>(a, (int)(n0 + blockIdx.x));
}

// Level-1 nodes that run alone (their order is folded afterwards).
template <int NB, typename S, bool ONE>
__global__ __launch_bounds__(kBfLevelThreads) void k_bf_level_list(BfArgs<S> a, const int *__restrict__ list,
                                                                   long long n0) {
    level_node_g<NB, S, ONE>(a, list[n0 + blockIdx.x]);
}

// Level 1 fused with the even/odd fold (Eqs. 13-14): one workgroup per unit
// {even node, odd node, first ring k0, slot}; both nodes cover the rings
// k0 .. k0+n-1 of one order, so q^even and q^odd of those rings meet in LDS
// and q(z) = q^e + q^o, q(-z) = q^e - q^o go straight to q.
constexpr int kBfFoldThreads = 2 * kBfLevelThreads;

template <int NB, typename S, bool ONE>
__global__ __launch_bounds__(kBfFoldThreads) void k_bf_level1_fold(BfArgs<S> a, const int4 *__restrict__ units,
                                                                   long long u0, int batch, int nbatch) {
    constexpr int NC = 2 * NB;
    extern __shared__ char lds_raw[];
    const int4 un = units[u0 + blockIdx.x];
    const int *nie = a.node_i + (size_t)un.x * kBfNodeInts;
    const int n = nie[2] + nie[4];
    S *uE = reinterpret_cast<S *>(lds_raw);  // even node: children 0 and 1, then the odd node's
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int par = w / (2 * kBfHalves), wc = w % (2 * kBfHalves);
    const int m = batch + un.w * nbatch, k0 = un.z;
    const int G = ONE ? 1 : a.G;
    for (int g = 0; g < G; g++) {
        if (g) __syncthreads();  // the previous group's fold has read LDS
        id_block<NB, S, ONE>(a, par ? un.y : un.x, wc & 1, wc >> 1, threadIdx.x & 63,
                             uE + (size_t)(2 * par + (wc & 1)) * n * NC, g * NC);
        __syncthreads();
        const int mb = a.map0 + g * NB;
        for (int e = threadIdx.x; e < n * NB; e += kBfFoldThreads) {
            const int c = e / NB, b = e % NB;
            const S *e0 = uE + c * NC + 2 * b, *e1 = e0 + (size_t)n * NC, *o0 = e1 + (size_t)n * NC,
                    *o1 = o0 + (size_t)n * NC;
            double er = (double)(e0[0] + e1[0]), ei = (double)(e0[1] + e1[1]);
            double orr = (double)(o0[0] + o1[0]), oi = (double)(o0[1] + o1[1]);
            if (m == 0) ei = oi = 0.0;  // real field: Im a_l0 is ignored
            const int k = k0 + c, ks = a.nrings - 1 - k;
            a.q[((size_t)k * (a.L + 1) + m) * a.nmaps + mb + b] = make_double2(er + orr, ei + oi);
            if (ks != k) a.q[((size_t)ks * (a.L + 1) + m) * a.nmaps + mb + b] = make_double2(er - orr, ei - oi);
        }
    }
}

// Fold of the listed slots of one batch: slot j holds order m = batch + j nbatch.
template <typename S>
__global__ __launch_bounds__(kBfThreads) void k_bf_fold(BfArgs<S> a, int batch, int nbatch, const int *__restrict__ slots,
                                                        int count) {
    const int K = a.K, NP = a.ES / 2;  // maps of the pass
    const long long e = (long long)blockIdx.x * kBfThreads + threadIdx.x;
    if (e >= (long long)count * K * NP) return;
    const int b = (int)(e % NP);
    const long long jk = e / NP;
    const int k = (int)(jk % K), j = slots[jk / K];
    const int m = batch + j * nbatch;
    const S *qe = a.ws + ((size_t)(2 * j) * K + k) * a.ES + 2 * b;
    const S *qo = a.ws + ((size_t)(2 * j + 1) * K + k) * a.ES + 2 * b;
    double er = (double)qe[0], ei = (double)qe[1], orr = (double)qo[0], oi = (double)qo[1];
    if (m == 0) ei = oi = 0.0;  // real field: Im a_l0 is ignored
    a.q[((size_t)k * (a.L + 1) + m) * a.nmaps + a.map0 + b] = make_double2(er + orr, ei + oi);
    const int ks = a.nrings - 1 - k;
    if (ks != k) a.q[((size_t)ks * (a.L + 1) + m) * a.nmaps + a.map0 + b] = make_double2(er - orr, ei - oi);
}

// ---- work-queue batches: one launch per stage for every request pass of
// one map-group width; item = {pass (argument block), index within the
// pass's plan}.  The bodies are the single-request kernels'.
template <int NB, typename S>
__global__ __launch_bounds__(kBfThreads) void k_bfq_residual(const BfArgs<S> *__restrict__ args,
                                                             const int2 *__restrict__ items, long long n) {
    __shared__ double stg_all[kBfThreads / 64][bf_res_stage_doubles<NB>()];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long j = (long long)blockIdx.x * (kBfThreads / 64) + w;
    if (j >= n) return;
    const int2 it = items[j];
    const BfArgs<S> a = args[__builtin_amdgcn_readfirstlane(it.x)];
    residual_piece<NB, S>(a, __builtin_amdgcn_readfirstlane(it.y), threadIdx.x & 63, stg_all[w], 0);
}

// items {pass, node}: level nodes, and level-1 nodes that run alone
template <int NB, typename S>
__global__ __launch_bounds__(kBfLevelThreads) void k_bfq_level(const BfArgs<S> *__restrict__ args,
                                                               const int2 *__restrict__ items) {
    const int2 it = items[blockIdx.x];
    const BfArgs<S> a = args[__builtin_amdgcn_readfirstlane(it.x)];
    level_node_g<NB, S, true>(a, __builtin_amdgcn_readfirstlane(it.y));
}

// items {pass, fused level-1 unit}
template <int NB, typename S>
__global__ __launch_bounds__(kBfFoldThreads) void k_bfq_level1_fold(const BfArgs<S> *__restrict__ args,
                                                                    const int2 *__restrict__ items) {
    constexpr int NC = 2 * NB;
    extern __shared__ char lds_raw[];
    const int2 it = items[blockIdx.x];
    const BfArgs<S> a = args[__builtin_amdgcn_readfirstlane(it.x)];
    const int4 un = a.f1_unit[__builtin_amdgcn_readfirstlane(it.y)];
    const int *nie = a.node_i + (size_t)un.x * kBfNodeInts;
    const int n = nie[2] + nie[4];
    S *uE = reinterpret_cast<S *>(lds_raw);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int par = w / (2 * kBfHalves), wc = w % (2 * kBfHalves);
    const int m = un.w, k0 = un.z;  // one order batch: slot j holds order j
    id_block<NB, S, true>(a, par ? un.y : un.x, wc & 1, wc >> 1, threadIdx.x & 63,
                          uE + (size_t)(2 * par + (wc & 1)) * n * NC, 0);
    __syncthreads();
    for (int e = threadIdx.x; e < n * NB; e += kBfFoldThreads) {
        const int c = e / NB, b = e % NB;
        const S *e0 = uE + c * NC + 2 * b, *e1 = e0 + (size_t)n * NC, *o0 = e1 + (size_t)n * NC,
                *o1 = o0 + (size_t)n * NC;
        double er = (double)(e0[0] + e1[0]), ei = (double)(e0[1] + e1[1]);
        double orr = (double)(o0[0] + o1[0]), oi = (double)(o0[1] + o1[1]);
        if (m == 0) ei = oi = 0.0;  // real field: Im a_l0 is ignored
        const int k = k0 + c, ks = a.nrings - 1 - k;
        a.q[((size_t)k * (a.L + 1) + m) * a.nmaps + a.map0 + b] = make_double2(er + orr, ei + oi);
        if (ks != k) a.q[((size_t)ks * (a.L + 1) + m) * a.nmaps + a.map0 + b] = make_double2(er - orr, ei - oi);
    }
}

// items {pass, block of kBfThreads fold elements}
template <typename S>
__global__ __launch_bounds__(kBfThreads) void k_bfq_fold(const BfArgs<S> *__restrict__ args,
                                                         const int2 *__restrict__ items) {
    const int2 it = items[blockIdx.x];
    const BfArgs<S> a = args[__builtin_amdgcn_readfirstlane(it.x)];
    const int K = a.K, NP = a.ES / 2;
    const long long e = (long long)__builtin_amdgcn_readfirstlane(it.y) * kBfThreads + threadIdx.x;
    if (e >= (long long)a.fold_count * K * NP) return;
    const int b = (int)(e % NP);
    const long long jk = e / NP;
    const int k = (int)(jk % K), j = a.fold_slot[jk / K];
    const int m = j;
    const S *qe = a.ws + ((size_t)(2 * j) * K + k) * a.ES + 2 * b;
    const S *qo = a.ws + ((size_t)(2 * j + 1) * K + k) * a.ES + 2 * b;
    double er = (double)qe[0], ei = (double)qe[1], orr = (double)qo[0], oi = (double)qo[1];
    if (m == 0) ei = oi = 0.0;
    a.q[((size_t)k * (a.L + 1) + m) * a.nmaps + a.map0 + b] = make_double2(er + orr, ei + oi);
    const int ks = a.nrings - 1 - k;
    if (ks != k) a.q[((size_t)ks * (a.L + 1) + m) * a.nmaps + a.map0 + b] = make_double2(er - orr, ei - oi);
}

template <int NB, typename S>
static hipError_t bfq_stage_nb(int stage, const void *args, const int2 *items, long long n, size_t lds, hipStream_t st) {
    const BfArgs<S> *ar = reinterpret_cast<const BfArgs<S> *>(args);
    constexpr int WPB = kBfThreads / 64;
    if (n <= 0) return hipSuccess;
    switch (stage) {
        case 0:
            hipLaunchKernelGGL((k_bfq_residual<NB, S>), dim3((unsigned)((n + WPB - 1) / WPB)), dim3(kBfThreads), 0, st, ar,
                               items, n);
            break;
        case 1:
            hipLaunchKernelGGL((k_bfq_level<NB, S>), dim3((unsigned)n), dim3(kBfLevelThreads), lds, st, ar, items);
            break;
        case 2:
            hipLaunchKernelGGL((k_bfq_level1_fold<NB, S>), dim3((unsigned)n), dim3(kBfFoldThreads), lds, st, ar, items);
            break;
        default:
            hipLaunchKernelGGL((k_bfq_fold<S>), dim3((unsigned)n), dim3(kBfThreads), 0, st, ar, items);
            break;
    }
    return hipGetLastError();
}

// One stage launch of a work-queue batch: stage 0 residual pieces, 1 level
// nodes (lds: widest column set), 2 fused level-1 units, 3 fold blocks.
hipError_t launch_bf_queue_stage(int stage, int nb, int fp32, const void *args, const int2 *items, long long n,
                                 size_t lds, hipStream_t st) {
    if (n > 0x7fffffffLL) return hipErrorInvalidValue;
    if (fp32) {
        switch (nb) {
            case 8: return bfq_stage_nb<8, float>(stage, args, items, n, lds, st);
            case 4: return bfq_stage_nb<4, float>(stage, args, items, n, lds, st);
            case 2: return bfq_stage_nb<2, float>(stage, args, items, n, lds, st);
            default: return bfq_stage_nb<1, float>(stage, args, items, n, lds, st);
        }
    }
    switch (nb) {
        case 8: return bfq_stage_nb<8, double>(stage, args, items, n, lds, st);
        case 4: return bfq_stage_nb<4, double>(stage, args, items, n, lds, st);
        case 2: return bfq_stage_nb<2, double>(stage, args, items, n, lds, st);
        default: return bfq_stage_nb<1, double>(stage, args, items, n, lds, st);
    }
}

// The argument block of one pass of a work-queue batch (G = 1, nb maps).
size_t bf_args_bytes(int fp32) { return fp32 ? sizeof(BfArgs<float>) : sizeof(BfArgs<double>); }
void bf_queue_args(const sht_plan_s *p, int nmaps, int map0, int nb, int fp32, const double *alm, double *q, void *ws,
                   void *out) {
    if (fp32) {
        BfArgs<float> a = bf_args<float>(p, nmaps, p->d_bf_T32, (float *)ws);
        a.alm = reinterpret_cast<const double2 *>(alm);
        a.q = reinterpret_cast<double2 *>(q);
        a.map0 = map0;
        a.ES = 2 * nb;
        a.G = 1;
        std::memcpy(out, &a, sizeof(a));
    } else {
        BfArgs<double> a = bf_args<double>(p, nmaps, p->d_bf_T, (double *)ws);
        a.alm = reinterpret_cast<const double2 *>(alm);
        a.q = reinterpret_cast<double2 *>(q);
        a.map0 = map0;
        a.ES = 2 * nb;
        a.G = 1;
        std::memcpy(out, &a, sizeof(a));
    }
}

// dynamic LDS of a level node / fused unit with n columns
size_t bf_level_lds_bytes(int n, int nb, int fp32) {
    return (size_t)n * 2 * (2 * nb * (fp32 ? sizeof(float) : sizeof(double)));
}

size_t bf_scratch_bytes(const sht_plan_s *p, int nmaps, int fp32) {
    return (size_t)p->bf.ws_entries * bf_entry_values(nmaps) * (fp32 ? sizeof(float) : sizeof(double));
}

// Records the caller's stage event (which = 0 before, 1 after) if given.
static void bf_event(void *const *ev, int stage, int which, hipStream_t st) {
    if (ev && ev[2 * stage + which]) (void)hipEventRecord((hipEvent_t)ev[2 * stage + which], st);
}

template <int NB, typename S, bool ONE>
static hipError_t launch_bf_nbg(const sht_plan_s *p, BfArgs<S> a, hipStream_t st, void *const *ev) {
    constexpr int WPB = kBfThreads / 64;
    const BflyPlan &b = p->bf;
    if (b.nbatch != 1) ev = nullptr;
    for (int bt = 0; bt < b.nbatch; bt++) {
        const long long t0 = b.batch_sub[bt], t1 = b.batch_sub[bt + 1];
        bf_event(ev, SHT_STAGE_BF_RESIDUAL, 0, st);
        for (int g = 0; g < a.G && t1 > t0; g++) {  // one launch per group of NB maps
            BfArgs<S> ag = a;
            ag.map0 = a.map0 + g * NB;
            hipLaunchKernelGGL((k_bf_residual<NB, S>), dim3((unsigned)((t1 - t0 + WPB - 1) / WPB)), dim3(kBfThreads), 0,
                               st, ag, t0, t1, g * 2 * NB);
        }
        bf_event(ev, SHT_STAGE_BF_RESIDUAL, 1, st);
        bf_event(ev, SHT_STAGE_BF_LEVELS, 0, st);
        const long long *lo = b.lv_off.data() + (size_t)bt * (kBfMaxLv + 1);
        for (int q = 0; q < kBfMaxLv - 1; q++) {  // levels >= 2
            const long long n0 = lo[q], n1 = lo[q + 1];
            if (n1 <= n0) continue;
            // LDS for the widest column set of this level only
            const size_t lds = bf_level_lds<NB, S>(b.lv_max_n[(size_t)bt * kBfMaxLv + q]);
            hipLaunchKernelGGL((k_bf_level<NB, S, ONE>), dim3((unsigned)(n1 - n0)), dim3(kBfLevelThreads), lds, st, a,
                               n0);
        }
        bf_event(ev, SHT_STAGE_BF_LEVELS, 1, st);
        // level 1: fused with the fold where both parities have levels
        const size_t lds1 = bf_level_lds<NB, S>(b.lv_max_n[(size_t)bt * kBfMaxLv + kBfMaxLv - 1]);
        const long long p0 = b.l1_off[bt], p1 = b.l1_off[bt + 1];
        if (p1 > p0)
            hipLaunchKernelGGL((k_bf_level_list<NB, S, ONE>), dim3((unsigned)(p1 - p0)), dim3(kBfLevelThreads), lds1, st, a,
                               p->d_bf_l1_plain, p0);
        const long long f0 = b.f1_off[bt], f1 = b.f1_off[bt + 1];
        if (f1 > f0)
            hipLaunchKernelGGL((k_bf_level1_fold<NB, S, ONE>), dim3((unsigned)(f1 - f0)), dim3(kBfFoldThreads), 2 * lds1, st,
                               a, reinterpret_cast<const int4 *>(p->d_bf_f1_unit), f0, bt, b.nbatch);
        const long long s0 = b.fold_off[bt], s1 = b.fold_off[bt + 1];
        const long long nf = (s1 - s0) * b.K * (a.ES / 2);
        if (nf > 0)
            hipLaunchKernelGGL((k_bf_fold<S>), dim3((unsigned)((nf + kBfThreads - 1) / kBfThreads)),
                               dim3(kBfThreads), 0, st, a, bt, b.nbatch, p->d_bf_fold_slot + s0, (int)(s1 - s0));
    }
    return hipGetLastError();
}

// The residual kernel over another task list (the interpolation form's node
// tasks): a.res_sub, res_lane, res_val and z2 describe the tasks; one launch
// for a pass of nb maps (G = 1).
hipError_t launch_node_phase(const sht_plan_s *p, int nb, BfArgs<double> a, long long npieces, hipStream_t st) {
    (void)p;
    constexpr int WPB = kBfThreads / 64;
    if (npieces <= 0) return hipSuccess;
    const dim3 grid((unsigned)((npieces + WPB - 1) / WPB));
    switch (nb) {
        case 4: hipLaunchKernelGGL((k_bf_residual<4, double>), grid, dim3(kBfThreads), 0, st, a, 0LL, npieces, 0); break;
        case 2: hipLaunchKernelGGL((k_bf_residual<2, double>), grid, dim3(kBfThreads), 0, st, a, 0LL, npieces, 0); break;
        default: hipLaunchKernelGGL((k_bf_residual<1, double>), grid, dim3(kBfThreads), 0, st, a, 0LL, npieces, 0); break;
    }
    return hipGetLastError();
}

template <int NB, typename S>
static hipError_t launch_bf_nb(const sht_plan_s *p, BfArgs<S> a, hipStream_t st, void *const *ev) {
    return a.G == 1 ? launch_bf_nbg<NB, S, true>(p, a, st, ev) : launch_bf_nbg<NB, S, false>(p, a, st, ev);
}

template <typename S>
static hipError_t launch_bf(const sht_plan_s *p, int nmaps, const double *alm, double *q, S *ws, const S *T,
                            hipStream_t st, void *const *ev) {
    BfArgs<S> a = bf_args<S>(p, nmaps, T, ws);
    a.alm = reinterpret_cast<const double2 *>(alm);
    a.q = reinterpret_cast<double2 *>(q);
    hipError_t e = hipSuccess;
    for (int b = 0; b < nmaps && e == hipSuccess;) {
        int nb, groups;
        bf_pass_shape(nmaps - b, &nb, &groups);
        a.map0 = b;
        a.G = groups;
        a.ES = 2 * nb * groups;
        switch (nb) {
            case 8: e = launch_bf_nb<8, S>(p, a, st, ev); break;
            case 4: e = launch_bf_nb<4, S>(p, a, st, ev); break;
            case 2: e = launch_bf_nb<2, S>(p, a, st, ev); break;
            default: e = launch_bf_nb<1, S>(p, a, st, ev); break;
        }
        b += nb * groups;
    }
    return e;
}

hipError_t launch_butterfly(const sht_plan_s *p, int nmaps, const double *alm, double *q, void *scratch,
                            int fp32, hipStream_t stream, void *const *stage_events) {
    if (fp32) return launch_bf<float>(p, nmaps, alm, q, (float *)scratch, p->d_bf_T32, stream, stage_events);
    return launch_bf<double>(p, nmaps, alm, q, (double *)scratch, p->d_bf_T, stream, stage_events);
}

}  // namespace sht
