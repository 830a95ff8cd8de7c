// Adjoint of the butterfly-compressed Legendre phase (Sec. 3.2 and App. A.1
// of the Wavemoth paper): g^t = Lambda ybar^t (Sec. 2.4 Eq. 12 transposed)
// runs the factorization backwards, per batch of orders:
//  1. level 1 takes ybar^even = ybar(z) + ybar(-z) and ybar^odd =
//     ybar(z) - ybar(-z) per north ring (Eqs. 13-14 transposed):
//     k_bf_unfold_level1 builds both for the two level-1 nodes of one order
//     and ring range in LDS and splits them at once; orders whose parities
//     split differently get their level-1 vectors from k_bf_unfold and run
//     k_bf_level_t over the listed level-1 nodes;
//  2. k_bf_level_t, level 2 and down: each pair node splits u into its
//     children, v_ch = A~_ch u (identity rows gather u, the dense part T U
//     runs on the matrix cores), so no two waves write one entry;
//  3. k_bf_residual_t: one wave per residual task regenerates the Legendre
//     values of its skeleton rings row by row, reduces sum_z P~(z) v(z) over
//     the wave with lane swaps and DPP, and adds the row's result to g with
//     one atomic per component (several tasks share a row block's rows, so
//     the order of those few addends, and the last bits of g, may vary from
//     run to run).
#include "butterfly_common.h"

namespace sht {

// Unfold of the listed slots of one batch: slot j (order m = batch + j
// nbatch) gets ybar^even and ybar^odd of every north ring in its level-1
// vectors (the equator once).
template <typename S>
__global__ __launch_bounds__(kBfThreads) void k_bf_unfold(BfArgs<S> a, int batch, int nbatch,
                                                          const int *__restrict__ slots, int count) {
    const int K = a.K, NP = a.ES / 2;  // maps of the pass
    const long long e = (long long)blockIdx.x * kBfThreads + threadIdx.x;
    if (e >= (long long)count * K * NP) return;
    const int b = (int)(e % NP);
    const long long jk = e / NP;
    const int k = (int)(jk % K), j = slots[jk / K];
    const int m = batch + j * nbatch;
    const int ks = a.nrings - 1 - k;
    const double2 yn = a.ybar[((size_t)k * (a.L + 1) + m) * a.nmaps + a.map0 + b];
    const double2 ys =
        ks != k ? a.ybar[((size_t)ks * (a.L + 1) + m) * a.nmaps + a.map0 + b] : make_double2(0.0, 0.0);
    S *qe = a.ws + ((size_t)(2 * j) * K + k) * a.ES + 2 * b;
    S *qo = a.ws + ((size_t)(2 * j + 1) * K + k) * a.ES + 2 * b;
    qe[0] = (S)(yn.x + ys.x);
    qe[1] = (S)(yn.y + ys.y);
    qo[0] = (S)(yn.x - ys.x);
    qo[1] = (S)(yn.y - ys.y);
}

// One ID block transposed (child ch of a pair node) on one wave:
//   v_ch = A~_ch u:  v[s] = u[perm s] + sum_d T[s][d] u[perm (k + d)].
// The dense part runs on the matrix cores with the skeleton rows s as the
// output rows (four 16-row tiles sharing each U operand) and the dense
// columns d as the reduction, kBfTJ K-steps per batch of loads.  With the
// transposed copy (TT, T^T row-major) lane (i, kq) of K-step j reads
// T^T[d0 + 4 j + kq][s0 + i], 16 consecutive entries per row as in the
// synthesis; otherwise it reads T[s0 + i][d0 + kBfTJ kq + j], kBfTJ
// contiguous entries of 16 different rows.
constexpr int kBfTJ = 2;  // K-steps per batch of loads in the transposed level

// NT 16-row tiles of skeleton rows s0 .. s0 + 16 NT - 1 of one transposed ID
// block (the tile count is a template parameter so that the products run
// back to back).  Columns d past nd get U = 0; rows past k hold clamped rows
// that are not stored.
template <int NT, int NB, bool TT, typename S>
__device__ __forceinline__ void split_tiles(const S *__restrict__ Tb, S *__restrict__ v, int ES, const S *u,
                                            const int16_t *pl, int kk, int nd, int s0, int lane) {
    constexpr int NC = 2 * NB;
    constexpr int DB = 4 * kBfTJ;  // dense columns per batch
    typedef typename Acc<S>::type acc_t;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int ic = min(i16, NC - 1);
    acc_t acc[NT];
#pragma unroll
    for (int tt = 0; tt < NT; tt++) acc[tt] = acc_t{0, 0, 0, 0};
    for (int d0 = 0; d0 < nd; d0 += DB) {
        S av[NT][kBfTJ], bv[kBfTJ];
#pragma unroll
        for (int j = 0; j < kBfTJ; j++) {
            const int d = TT ? d0 + 4 * j + k4 : d0 + kBfTJ * k4 + j, dc = min(d, nd - 1);
            bv[j] = u[pl[kk + dc] * NC + ic] * (S)(d < nd);
#pragma unroll
            for (int tt = 0; tt < NT; tt++) {
                const int sr = min(s0 + 16 * tt + i16, kk - 1);
                av[tt][j] = Tb[TT ? (unsigned)(dc * kk + sr) : (unsigned)(sr * nd + dc)];
            }
        }
#pragma unroll
        for (int j = 0; j < kBfTJ; j++)
#pragma unroll
            for (int tt = 0; tt < NT; tt++) acc[tt] = mfma_16x16x4(av[tt][j], bv[j], acc[tt]);
    }
#pragma unroll
    for (int tt = 0; tt < NT; tt++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int sr = s0 + 16 * tt + acc_row<S>(k4, r);
            if (sr < kk && i16 < NC) v[sr * ES + i16] = acc[tt][r] + u[pl[sr] * NC + i16];
        }
}

template <int NB, bool TT, typename S, bool ONE>
__device__ __forceinline__ void id_block_t(const BfArgs<S> &a, int node, int ch, int half, int lane, const S *u,
                                           const int16_t *pl, int col) {
    constexpr int TPW = 4 / kBfHalves;  // 16-row tiles per wave
    const int *ni = a.node_i + (size_t)node * kBfNodeInts;
    const int kk = ni[2 + ch], nd = ni[4 + ch];
    const int ES = ONE ? 2 * NB : a.ES;  // one group per pass: the stride is a constant
    S *__restrict__ v = a.ws + (size_t)ni[ch] * ES + col;
    const long long toff = (long long)(unsigned)ni[12 + 2 * ch] | ((long long)ni[13 + 2 * ch] << 32);
    const S *__restrict__ Tb = a.T + toff;
    for (int s00 = 0; s00 < kk; s00 += 64) {
        const int ntile = min(TPW, min(4, (kk - s00 + 15) >> 4) - half * TPW);  // tiles of this wave
        const int s0 = s00 + 16 * TPW * half;
        switch (ntile) {
            case 1: split_tiles<1, NB, TT, S>(Tb, v, ES, u, pl, kk, nd, s0, lane); break;
            case 2: split_tiles<2, NB, TT, S>(Tb, v, ES, u, pl, kk, nd, s0, lane); break;
            case 3: split_tiles<3, NB, TT, S>(Tb, v, ES, u, pl, kk, nd, s0, lane); break;
            case 4: split_tiles<4, NB, TT, S>(Tb, v, ES, u, pl, kk, nd, s0, lane); break;
            default: break;
        }
    }
}

// LDS of one transposed pair node with n columns: u (n entries of 2 NB
// values) and both children's column permutations (2 n int16).
template <int NB, typename S>
inline size_t bf_level_t_lds(int n) {
    return (size_t)n * (2 * NB * sizeof(S) + 2 * sizeof(int16_t));
}

// One workgroup of 2 kBfHalves waves per pair node: per group of NB maps,
// u is staged in LDS, then wave w writes half w / 2 of the rows of child
// w % 2's vector.
template <int NB, bool TT, typename S, bool ONE>
__device__ __forceinline__ void level_node_tg(const BfArgs<S> &a, int node) {
    constexpr int NC = 2 * NB;
    extern __shared__ char lds_raw[];
    S *u = reinterpret_cast<S *>(lds_raw);
    const int *ni = a.node_i + (size_t)node * kBfNodeInts;
    const int n = ni[2] + ni[4];
    int16_t *pl = reinterpret_cast<int16_t *>(u + (size_t)n * NC);
    const int ES = ONE ? NC : a.ES, G = ONE ? 1 : a.G;
    const S *__restrict__ in = a.ws + (size_t)ni[6] * ES;
    const int16_t *__restrict__ pg = a.perm + ni[7];
    for (int e = threadIdx.x; e < 2 * n; e += kBfLevelThreads) pl[e] = pg[e];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int g = 0; g < G; g++) {
        if (g) __syncthreads();  // the previous group's splits have read u
        if (ONE) {
            for (int e = threadIdx.x; e < n * NC; e += kBfLevelThreads) u[e] = in[e];
        } else {
            for (int e = threadIdx.x; e < n * NC; e += kBfLevelThreads) u[e] = in[(size_t)(e / NC) * ES + g * NC + e % NC];
        }
        __syncthreads();
        id_block_t<NB, TT, S, ONE>(a, node, w & 1, w >> 1, threadIdx.x & 63, u, pl + (w & 1) * n, g * NC);
    }
}



// ONE: the pass has a single group of maps (separate instantiations, so the
// common case keeps its constant strides and its register count).
template <int NB, bool TT, typename S, bool ONE>
__global__ __launch_bounds__(kBfLevelThreads) void k_bf_level_t(BfArgs<S> a, long long n0) {
    level_node_tg<NB, TT, S, ONE>(a, (int)(n0 + blockIdx.x));
}

// Level-1 nodes that run alone (their order was unfolded beforehand).
template <int NB, bool TT, typename S, bool ONE>
__global__ __launch_bounds__(kBfLevelThreads) void k_bf_level_t_list(BfArgs<S> a, const int *__restrict__ list,
                                                                     long long n0) {
    level_node_tg<NB, TT, S, ONE>(a, list[n0 + blockIdx.x]);
}

// Unfold fused with level 1 (Eqs. 13-14 transposed): one workgroup per unit
// {even node, odd node, first ring k0, slot}; both nodes cover the rings
// k0 .. k0+n-1 of one order, so ybar^even and ybar^odd of those rings are
// built in LDS from the two hemispheres' ybar and split by both nodes at once.
constexpr int kBfUnfoldThreads = 2 * kBfLevelThreads;

template <int NB, bool TT, typename S, bool ONE>
__global__ __launch_bounds__(kBfUnfoldThreads) void k_bf_unfold_level1(BfArgs<S> a, const int4 *__restrict__ units,
                                                                       long long u0, int batch, int nbatch) {
    constexpr int NC = 2 * NB;
    extern __shared__ char lds_raw[];
    const int4 un = units[u0 + blockIdx.x];
    const int *nie = a.node_i + (size_t)un.x * kBfNodeInts;
    const int n = nie[2] + nie[4];
    S *uE = reinterpret_cast<S *>(lds_raw);
    S *uO = uE + (size_t)n * NC;
    int16_t *pl = reinterpret_cast<int16_t *>(uO + (size_t)n * NC);  // even node's 2n entries, then odd's
    const int16_t *__restrict__ pe = a.perm + nie[7];
    const int16_t *__restrict__ po = a.perm + a.node_i[(size_t)un.y * kBfNodeInts + 7];
    for (int e = threadIdx.x; e < 4 * n; e += kBfUnfoldThreads) pl[e] = e < 2 * n ? pe[e] : po[e - 2 * n];
    const int m = batch + un.w * nbatch, k0 = un.z;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int par = w / (2 * kBfHalves), wc = w % (2 * kBfHalves);
    const int G = ONE ? 1 : a.G;
    for (int g = 0; g < G; g++) {
        if (g) __syncthreads();  // the previous group's splits have read uE and uO
        const int mb = a.map0 + g * NB;
        for (int e = threadIdx.x; e < n * NB; e += kBfUnfoldThreads) {
            const int c = e / NB, b = e % NB;
            const int k = k0 + c, ks = a.nrings - 1 - k;
            const double2 yn = a.ybar[((size_t)k * (a.L + 1) + m) * a.nmaps + mb + b];
            const double2 ys =
                ks != k ? a.ybar[((size_t)ks * (a.L + 1) + m) * a.nmaps + mb + b] : make_double2(0.0, 0.0);
            uE[c * NC + 2 * b] = (S)(yn.x + ys.x);
            uE[c * NC + 2 * b + 1] = (S)(yn.y + ys.y);
            uO[c * NC + 2 * b] = (S)(yn.x - ys.x);
            uO[c * NC + 2 * b + 1] = (S)(yn.y - ys.y);
        }
        __syncthreads();
        id_block_t<NB, TT, S, ONE>(a, par ? un.y : un.x, wc & 1, wc >> 1, threadIdx.x & 63, par ? uO : uE,
                                   pl + (2 * par + (wc & 1)) * n, g * NC);
    }
}

// Lane exchanges for the wave reductions.  permlane32_swap(a, b) leaves
// a = [a lanes 0-31, b lanes 0-31] and b = [a lanes 32-63, b lanes 32-63];
// permlane16_swap does the same with rows of 16 (a keeps its even rows and
// b's even rows, b gets the odd rows of both), as measured on gfx950.
__device__ __forceinline__ void swap32(double &a, double &b) {
    const long long ia = __builtin_bit_cast(long long, a), ib = __builtin_bit_cast(long long, b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ia, (unsigned)ib, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
    a = __builtin_bit_cast(double, ((long long)hi[0] << 32) | (long long)lo[0]);
    b = __builtin_bit_cast(double, ((long long)hi[1] << 32) | (long long)lo[1]);
}
__device__ __forceinline__ void swap16(double &a, double &b) {
    const long long ia = __builtin_bit_cast(long long, a), ib = __builtin_bit_cast(long long, b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ia, (unsigned)ib, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
    a = __builtin_bit_cast(double, ((long long)hi[0] << 32) | (long long)lo[0]);
    b = __builtin_bit_cast(double, ((long long)hi[1] << 32) | (long long)lo[1]);
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// One in-row stage at lane distance given by CTRL (a DPP pattern pairing
// lanes that differ in bit BIT): with h > 0 it halves the values (value j
// stays where the bit is clear, value j + h where it is set), with h = 0 it
// adds the partner's single value.
template <int CTRL, int BIT, int N>
__device__ __forceinline__ void row_stage(double (&x)[N], int h, int lane) {
    const bool hi = (lane >> BIT) & 1;
    if (h == 0) {
        x[0] += dpp_mov<CTRL>(x[0]);
        return;
    }
#pragma unroll
    for (int j = 0; j < N / 2; j++) {
        if (j >= h) break;
        const double keep = hi ? x[j + h] : x[j], send = hi ? x[j] : x[j + h];
        x[j] = keep + dpp_mov<CTRL>(send);
    }
}

// Sum of x[c] over the 64 lanes of a wave for N = 2^A values per lane
// (N <= 16): afterwards value c = lane >> (6 - A) is complete in every lane
// of its group.  Lane distances 32 and 16 use lane swaps (each pair of
// values costs two swaps and one add), 8, 4, 2, 1 use DPP.
template <int N>
__device__ __forceinline__ double wave_transpose_sum(double (&x)[N], int lane) {
    static_assert(N == 1 || N == 2 || N == 4 || N == 8 || N == 16, "value count");
    int h = N / 2;
    if (h > 0) {
#pragma unroll
        for (int j = 0; j < N / 2; j++) {
            swap32(x[j], x[j + N / 2]);
            x[j] += x[j + N / 2];
        }
    } else {
        double y = x[0];
        swap32(x[0], y);
        x[0] += y;
    }
    h /= 2;
    if (h > 0) {
#pragma unroll
        for (int j = 0; j < N / 4; j++) {
            swap16(x[j], x[j + N / 4]);
            x[j] += x[j + N / 4];
        }
    } else {
        double y = x[0];
        swap16(x[0], y);
        x[0] += y;
    }
    h /= 2;
    row_stage<0x128, 3>(x, h, lane);  // row_ror:8
    h /= 2;
    row_stage<0x141, 2>(x, h, lane);  // row_half_mirror
    h /= 2;
    row_stage<0x4E, 1>(x, h, lane);   // quad_perm [2,3,0,1]
    h /= 2;
    row_stage<0xB1, 0>(x, h, lane);   // quad_perm [1,0,3,2]
    return x[0];
}

// One transposed residual task on one wave: R rings per lane, rows
// [imin, iend) of parity t; each row's sum over the task's rings goes to g.
template <int NB, int R, typename S>
__device__ __forceinline__ void residual_task_t(const BfArgs<S> &a, long long tk, int lane, int t, int imin,
                                                int iend, int nl, int outb, int m, c_double *cfs, int col0) {
    constexpr int NC = 2 * NB;
    constexpr int A = NC == 2 ? 1 : NC == 4 ? 2 : NC == 8 ? 3 : 4;
    int i0[R];
    double z2[R], v0[R], v1[R], P0[R], P1[R], w[R][NC];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const size_t li = (size_t)tk * kBfTaskRings + r * 64 + lane;
        const int2 ln = a.res_lane[li];
        const double2 sv = a.res_val[li];
        i0[r] = ln.y;
        z2[r] = a.z2[ln.x];
        v0[r] = sv.x;
        v1[r] = sv.y;
        P0[r] = P1[r] = 0.0;
        const int j = r * 64 + lane;
#pragma unroll
        for (int c = 0; c < NC; c++) w[r][c] = j < nl ? (double)a.ws[((size_t)outb + j) * a.ES + col0 + c] : 0.0;
    }
    const size_t aoff = (size_t)m * (2 * a.L + 3 - m) / 2;
    // component c = 2 b + (re, im) of row i lives at gb[i * 4 nmaps + c]
    double *gb = a.g + 2 * ((aoff + t) * a.nmaps + a.map0);
    const size_t gstride = 4 * (size_t)a.nmaps;
    const int c_own = lane >> (6 - A);
    const bool writer = (lane & ((1 << (6 - A)) - 1)) == 0 && !(m == 0 && (c_own & 1));
    auto step = [&](int i) {
        c_double *e = cfs + 4 * (t + 2 * i + 2);
        const double eb = e[0], eab = e[1], eg = e[2];
        double part[NC];
#pragma unroll
        for (int c = 0; c < NC; c++) part[c] = 0.0;
#pragma unroll
        for (int r = 0; r < R; r++) {
#pragma unroll
            for (int c = 0; c < NC; c++) part[c] = __builtin_fma(P0[r], w[r][c], part[c]);
            const double P2 = __builtin_fma(__builtin_fma(z2[r], eb, eab), P1[r], eg * P0[r]);
            P0[r] = P1[r];
            P1[r] = P2;
        }
        const double tot = wave_transpose_sum<NC>(part, lane);
        if (writer) atomicAdd(gb + (size_t)i * gstride + c_own, tot);
    };
    for (int c = imin; c < iend;) {
#pragma unroll
        for (int r = 0; r < R; r++)
            if (i0[r] == c) {
                P0[r] = v0[r];
                P1[r] = v1[r];
            }
        const int ce = min(iend, (c & ~(kChunk - 1)) + kChunk);
        if (ce - c == kChunk) {
#pragma unroll
            for (int u = 0; u < kChunk; u++) step(c + u);
        } else {
            for (int i = c; i < ce; i++) step(i);
        }
        c = ce;
    }
}

template <int NB, typename S>
__global__ __launch_bounds__(kBfThreads) void k_bf_residual_t(BfArgs<S> a, long long t0, long long t1, int col0) {
    const int lane = threadIdx.x & 63;
    const long long tk = t0 + (long long)blockIdx.x * (kBfThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tk >= t1) return;
    const int4 h = a.res_task[2 * tk], h2 = a.res_task[2 * tk + 1];
    const int t = __builtin_amdgcn_readfirstlane(h.x), imin = __builtin_amdgcn_readfirstlane(h.y);
    const int iend = __builtin_amdgcn_readfirstlane(h.z), nl = __builtin_amdgcn_readfirstlane(h.w);
    const int outb = __builtin_amdgcn_readfirstlane(h2.x), m = __builtin_amdgcn_readfirstlane(h2.y);
    c_double *cfs = (c_double *)(a.coef + 4 * a.coef_off[m]);
    if constexpr (kBfTaskRings > 192) {
        if (nl > 192) return residual_task_t<NB, 4>(a, tk, lane, t, imin, iend, nl, outb, m, cfs, col0);
    }
    if constexpr (kBfTaskRings > 128) {
        if (nl > 128) return residual_task_t<NB, 3>(a, tk, lane, t, imin, iend, nl, outb, m, cfs, col0);
    }
    if constexpr (kBfTaskRings > 64) {
        if (nl > 64) return residual_task_t<NB, 2>(a, tk, lane, t, imin, iend, nl, outb, m, cfs, col0);
    }
    residual_task_t<NB, 1>(a, tk, lane, t, imin, iend, nl, outb, m, cfs, col0);
}

// g = 0 over the nalm rows of maps [map0, map0 + nb) (a kernel, not a
// memset, so that the adjoint can be captured into a graph).
__global__ __launch_bounds__(kBfThreads) void k_bf_zero(double *g, long long nalm, int nmaps, int map0, int nb) {
    const long long e = (long long)blockIdx.x * kBfThreads + threadIdx.x;
    if (e >= nalm * nb * 2) return;
    const long long row = e / (2 * nb);
    const int rest = (int)(e % (2 * nb));
    g[2 * (row * nmaps + map0) + rest] = 0.0;
}

template <int NB, bool TT, typename S, bool ONE>
static hipError_t launch_bf_adj_nbg(const sht_plan_s *p, BfArgs<S> a, hipStream_t st) {
    constexpr int WPB = kBfThreads / 64;
    const BflyPlan &b = p->bf;
    const long long nalm = (long long)(p->L + 1) * (p->L + 2) / 2;
    const int np = NB * a.G;  // maps of the pass
    hipLaunchKernelGGL(k_bf_zero, dim3((unsigned)((nalm * np * 2 + kBfThreads - 1) / kBfThreads)), dim3(kBfThreads), 0,
                       st, a.g, nalm, a.nmaps, a.map0, np);
    for (int bt = 0; bt < b.nbatch; bt++) {
        // level 1: fused with the unfold where both parities have levels
        const long long s0 = b.fold_off[bt], s1 = b.fold_off[bt + 1];
        const long long nf = (s1 - s0) * b.K * np;
        if (nf > 0)
            hipLaunchKernelGGL((k_bf_unfold<S>), dim3((unsigned)((nf + kBfThreads - 1) / kBfThreads)),
                               dim3(kBfThreads), 0, st, a, bt, b.nbatch, p->d_bf_fold_slot + s0, (int)(s1 - s0));
        const size_t lds1 = bf_level_t_lds<NB, S>(b.lv_max_n[(size_t)bt * kBfMaxLv + kBfMaxLv - 1]);
        const long long p0 = b.l1_off[bt], p1 = b.l1_off[bt + 1];
        if (p1 > p0)
            hipLaunchKernelGGL((k_bf_level_t_list<NB, TT, S, ONE>), dim3((unsigned)(p1 - p0)), dim3(kBfLevelThreads), lds1, st,
                               a, p->d_bf_l1_plain, p0);
        const long long f0 = b.f1_off[bt], f1 = b.f1_off[bt + 1];
        if (f1 > f0)
            hipLaunchKernelGGL((k_bf_unfold_level1<NB, TT, S, ONE>), dim3((unsigned)(f1 - f0)), dim3(kBfUnfoldThreads), 2 * lds1,
                               st, a, reinterpret_cast<const int4 *>(p->d_bf_f1_unit), f0, bt, b.nbatch);
        const long long *lo = b.lv_off.data() + (size_t)bt * (kBfMaxLv + 1);
        for (int q = kBfMaxLv - 2; q >= 0; q--) {  // levels >= 2
            const long long n0 = lo[q], n1 = lo[q + 1];
            if (n1 <= n0) continue;
            const size_t lds = bf_level_t_lds<NB, S>(b.lv_max_n[(size_t)bt * kBfMaxLv + q]);
            hipLaunchKernelGGL((k_bf_level_t<NB, TT, S, ONE>), dim3((unsigned)(n1 - n0)), dim3(kBfLevelThreads), lds, st, a,
                               n0);
        }
        const long long t0 = b.batch_task[bt], t1 = b.batch_task[bt + 1];
        for (int g = 0; g < a.G && t1 > t0; g++) {  // one launch per group of NB maps
            BfArgs<S> ag = a;
            ag.map0 = a.map0 + g * NB;
            hipLaunchKernelGGL((k_bf_residual_t<NB, S>), dim3((unsigned)((t1 - t0 + WPB - 1) / WPB)),
                               dim3(kBfThreads), 0, st, ag, t0, t1, g * 2 * NB);
        }
    }
    return hipGetLastError();
}

template <int NB, bool TT, typename S>
static hipError_t launch_bf_adj_nb(const sht_plan_s *p, BfArgs<S> a, hipStream_t st) {
    return a.G == 1 ? launch_bf_adj_nbg<NB, TT, S, true>(p, a, st) : launch_bf_adj_nbg<NB, TT, S, false>(p, a, st);
}

template <typename S>
static hipError_t launch_bf_adj(const sht_plan_s *p, int nmaps, const double *ybar, double *g, S *ws, const S *T,
                                const S *Tt, hipStream_t st) {
    BfArgs<S> a = bf_args<S>(p, nmaps, Tt ? Tt : T, ws);
    a.ybar = reinterpret_cast<const double2 *>(ybar);
    a.g = g;
    hipError_t e = hipSuccess;
    for (int b = 0; b < nmaps && e == hipSuccess;) {
        int nb, groups;
        bf_pass_shape(nmaps - b, &nb, &groups);
        a.map0 = b;
        a.G = groups;
        a.ES = 2 * nb * groups;
        if (Tt) {
            switch (nb) {
                case 8: e = launch_bf_adj_nb<8, true, S>(p, a, st); break;
                case 4: e = launch_bf_adj_nb<4, true, S>(p, a, st); break;
                case 2: e = launch_bf_adj_nb<2, true, S>(p, a, st); break;
                default: e = launch_bf_adj_nb<1, true, S>(p, a, st); break;
            }
        } else {
            switch (nb) {
                case 8: e = launch_bf_adj_nb<8, false, S>(p, a, st); break;
                case 4: e = launch_bf_adj_nb<4, false, S>(p, a, st); break;
                case 2: e = launch_bf_adj_nb<2, false, S>(p, a, st); break;
                default: e = launch_bf_adj_nb<1, false, S>(p, a, st); break;
            }
        }
        b += nb * groups;
    }
    return e;
}

hipError_t launch_butterfly_adjoint(const sht_plan_s *p, int nmaps, const double *ybar, double *g, void *scratch,
                                    int fp32, hipStream_t stream) {
    if (fp32) return launch_bf_adj<float>(p, nmaps, ybar, g, (float *)scratch, p->d_bf_T32, p->d_bf_Tt32, stream);
    return launch_bf_adj<double>(p, nmaps, ybar, g, (double *)scratch, p->d_bf_T, p->d_bf_Tt, stream);
}

// Transposed copy of every interpolation block: child ch of a pair node keeps
// its kk x nd matrix T row-major at toff; Tt receives the nd x kk transpose
// at the same offset.  One workgroup per (node, child).
template <typename S>
__global__ __launch_bounds__(kBfThreads) void k_bf_transpose_blocks(const int *__restrict__ node_i,
                                                                    const S *__restrict__ T, S *__restrict__ Tt) {
    const int *ni = node_i + (size_t)(blockIdx.x >> 1) * kBfNodeInts;
    const int ch = blockIdx.x & 1;
    const int kk = ni[2 + ch], nd = ni[4 + ch];
    const long long toff = (long long)(unsigned)ni[12 + 2 * ch] | ((long long)ni[13 + 2 * ch] << 32);
    const int n = kk * nd;
    for (int f = threadIdx.x; f < n; f += kBfThreads) {
        const int d = f / kk, s = f - d * kk;
        Tt[toff + f] = T[toff + (long long)s * nd + d];
    }
}

hipError_t bf_store_transposed(sht_plan_s *p, size_t nT, size_t nnodes, size_t *bytes) {
    const size_t n = std::max<size_t>(nT, 1);
    if (2 * nnodes > 0xFFFFFFFFull) return hipErrorInvalidValue;
    hipError_t e = hipMalloc((void **)&p->d_bf_Tt, n * sizeof(double));
    if (e != hipSuccess) return e;
    *bytes += n * sizeof(double);
    if (nnodes)
        hipLaunchKernelGGL(k_bf_transpose_blocks<double>, dim3((unsigned)(2 * nnodes)), dim3(kBfThreads), 0, 0,
                           p->d_bf_node_i, p->d_bf_T, p->d_bf_Tt);
    if (p->d_bf_T32) {
        e = hipMalloc((void **)&p->d_bf_Tt32, n * sizeof(float));
        if (e != hipSuccess) return e;
        *bytes += n * sizeof(float);
        if (nnodes)
            hipLaunchKernelGGL(k_bf_transpose_blocks<float>, dim3((unsigned)(2 * nnodes)), dim3(kBfThreads), 0, 0,
                               p->d_bf_node_i, p->d_bf_T32, p->d_bf_Tt32);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e;
}

}  // namespace sht
