// Adjoint Legendre transform, for gfx950: the transpose of the Legendre
// phase of Sec. 2.4 Eq. 12 (the paper's backward Legendre transform of
// Sec. 3 Eq. 18 without quadrature weights), with the even/odd ring
// symmetry of Eqs. 13-14 applied in reverse:
//
//   g_lm = sum_{north k} P~_l^m(z_k) ybar^t_m(z_k),   t = (l - m) mod 2,
//   ybar^even(z) = ybar(z) + ybar(-z),  ybar^odd(z) = ybar(z) - ybar(-z)
//
// (the equator ring counts once).  The recurrence runs along l for every
// ring, but the outputs are indexed by l and summed over rings, so one
// workgroup owns one order m and a block of rings, each thread running the
// two-step recurrence (App. A.2 Eq. A2) for its rings.  Rings nearest the
// poles run the recurrence in double-double arithmetic in their own launch
// (k_legendre_adj: per-step partial sums over a thread's rings, added
// through double-buffered LDS), writing g; the FP64 ring blocks then add
// their share to g in place, launch after launch (k_legendre_adj_mf: the sum
// over rings as FP64 MFMA products of Legendre tiles with the ring phases).
// Every sum runs in a fixed order: deterministic, no atomics, no partial-sum
// workspace.
#include "internal.h"

namespace sht {

struct AdjArgs {
    const double *__restrict__ z2_hi;
    const double *__restrict__ z2_lo;
    const long long *__restrict__ coef_off;
    const double *__restrict__ coef_hi;
    const double *__restrict__ coef_lo;
    const int *__restrict__ start_idx;
    const double *__restrict__ start_val;
    const double *__restrict__ start_lo;
    const int *__restrict__ grp_lo;
    const int *__restrict__ grp_hi;
    const double2 *__restrict__ ybar;  // [ring][m][nmaps]
    double *__restrict__ g;            // [nalm][nmaps] complex
    int L, nrings, n_north, np, n_dd_pad, ng;
    int nmaps, map0;
    int k0, k1;        // north rings [k0, k1) handled by this launch
    int accumulate;    // 0: write g, 1: add to g
};

struct dd2 {
    double h, l;
};

#pragma clang fp contract(off)
__device__ __forceinline__ dd2 two_sum2(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ dd2 fast_two_sum2(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}
__device__ __forceinline__ dd2 dd2_mul(dd2 a, dd2 b) {
    double p = a.h * b.h;
    double e = __builtin_fma(a.h, b.h, -p);
    e = __builtin_fma(a.h, b.l, e);
    e = __builtin_fma(a.l, b.h, e);
    return fast_two_sum2(p, e);
}
__device__ __forceinline__ dd2 dd2_add(dd2 a, dd2 b) {
    dd2 s = two_sum2(a.h, b.h);
    double e = s.l + (a.l + b.l);
    return fast_two_sum2(s.h, e);
}
#pragma clang fp contract(on)

// Lane shuffle of a double within a row of 16 lanes (DPP control CTRL).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over each row of 16 lanes, every lane of the row receiving the total:
// pairs, quads, mirrored quads, mirrored halves.  Partners add the same two
// numbers, so the result is the same in every lane.
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    return v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// T = 256 threads, R rings per thread (rings k0 + tid*R + r, so each wave
// holds a contiguous block of rings), NB maps per pass.  A group of G chain
// steps (G * 4 * NB = 16 outputs) is written to one of two LDS buffers as
// per-thread partial sums red[G][4*NB][T]; after one barrier, 16 lanes per
// output add 16 partials each and finish with a 16-lane DPP tree, while the
// next group fills the other buffer.  Outputs already in g (accumulating
// launches) are fetched one group ahead.  The recurrence coefficients of the
// order stream through LDS in blocks of kAdjCB steps, each block fetched from
// memory two blocks ahead of its use, so that the chain never waits on HBM.
constexpr int kAdjCB = 32;  // chain steps per LDS coefficient block

template <int T, int R, int NB, bool DD>
__global__ __launch_bounds__(T) void k_legendre_adj(AdjArgs a) {
    static_assert(T == 256, "the reduction maps 16 outputs x 16 slices onto 256 threads");
    constexpr int NV = 4 * NB;     // (parity, map, re/im) components per step
    constexpr int G = 16 / NV;     // chain steps per LDS group
    constexpr int SL = T / 16;     // partial-sum slices per output
    constexpr int PS = T / SL;     // partials added by one slice
    constexpr int CW = 8;          // doubles per step and table: even B, AB, G, pad, odd B, AB, G, pad
    constexpr int CE = kAdjCB * CW / T;  // table entries per thread and block
    static_assert(kAdjCB % G == 0 && kAdjCB > G && CE >= 1, "coefficient block shape");
    extern __shared__ double red[];
    constexpr int GO = kAdjCB / G * 16;  // outputs per coefficient block
    static_assert(GO <= T, "one staged output per thread");
    __shared__ double cbuf[2][(DD ? 2 : 1) * kAdjCB * CW];
    __shared__ double gbuf_acc[2][GO];  // outputs already in g, for accumulating launches
    const int m = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int L = a.L;
    const int n0 = (L - m) / 2 + 1;
    const int n1 = (L - m >= 1) ? (L - m - 1) / 2 + 1 : 0;
    const size_t aoff = (size_t)m * (2 * L + 3 - m) / 2;

    // chain range over the groups of this launch's rings
    __shared__ int s_lo, s_hi;
    if (tid == 0) {
        int lo = kDead, hi = -1;
        for (int gr = a.k0 / kLanes; gr < (a.k1 + kLanes - 1) / kLanes; gr++) {
            lo = min(lo, a.grp_lo[(size_t)m * a.ng + gr]);
            hi = max(hi, a.grp_hi[(size_t)m * a.ng + gr]);
        }
        s_lo = lo;
        s_hi = hi;
    }
    __syncthreads();
    const int lo = s_lo, hi = s_hi;

    auto gaddr = [&](int l, int b, int ri) { return a.g + 2 * ((aoff + l - m) * a.nmaps + a.map0 + b) + ri; };

    if (lo >= n0) {  // every chain of these rings stays below the cutoff
        if (!a.accumulate)
            for (int e = tid; e < (L - m + 1) * NB * 2; e += T) *gaddr(m + e / (NB * 2), (e / 2) % NB, e % 2) = 0.0;
        return;
    }

    int k[R];
    bool val[R];
    double z2h[R], z2l[R];
    int sid[R][2];
    dd2 st0[R][2], st1[R][2], p0[R][2], p1[R][2];
    double yer[R][NB], yei[R][NB], yor[R][NB], yoi[R][NB];
    int wlo = kDead;
#pragma unroll
    for (int r = 0; r < R; r++) {
        k[r] = a.k0 + tid * R + r;
        val[r] = k[r] < a.k1 && k[r] < a.n_north;
        const int kk = val[r] ? k[r] : a.k0;
        z2h[r] = a.z2_hi[kk];
        z2l[r] = DD ? a.z2_lo[kk] : 0.0;
#pragma unroll
        for (int t = 0; t < 2; t++) {
            const size_t row = (size_t)(2 * m + t);
            sid[r][t] = val[r] ? a.start_idx[row * a.np + kk] : kDead;
            wlo = min(wlo, sid[r][t]);
            st0[r][t].h = a.start_val[(row * 2 + 0) * a.np + kk];
            st1[r][t].h = a.start_val[(row * 2 + 1) * a.np + kk];
            st0[r][t].l = DD ? a.start_lo[(row * 2 + 0) * a.n_dd_pad + kk] : 0.0;
            st1[r][t].l = DD ? a.start_lo[(row * 2 + 1) * a.n_dd_pad + kk] : 0.0;
            p0[r][t] = {0.0, 0.0};
            p1[r][t] = {0.0, 0.0};
        }
        // unfold the ring and its mirror into even/odd parts
        const int ks = a.nrings - 1 - kk;
        const double2 *yn = a.ybar + ((size_t)kk * (a.L + 1) + m) * a.nmaps + a.map0;
        const double2 *ys = a.ybar + ((size_t)ks * (a.L + 1) + m) * a.nmaps + a.map0;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            double2 vn = val[r] ? yn[b] : make_double2(0.0, 0.0);
            double2 vs = (val[r] && ks != kk) ? ys[b] : make_double2(0.0, 0.0);
            yer[r][b] = vn.x + vs.x;
            yei[r][b] = vn.y + vs.y;
            yor[r][b] = vn.x - vs.x;
            yoi[r][b] = vn.y - vs.y;
        }
    }
    // first chain step at which any ring of this wave is alive
    wlo = __builtin_amdgcn_readfirstlane(wave_min(wlo));

    // coefficient blocks: block j holds chain steps lo + j*kAdjCB + s, s < kAdjCB,
    // as the table entries 2*step + 2 (even chain) and 2*step + 3 (odd chain);
    // steps past n0 are not fetched (the table is padded only a few steps)
    const long long cbase = a.coef_off[m];
    const double *__restrict__ chd = a.coef_hi + 4 * cbase;
    const double *__restrict__ cld = a.coef_lo + 4 * cbase;
    // staged outputs: thread tid < GO holds output tid % 16 of group tid / 16
    const int so = tid % 16, sv = so % NV, sg = so / NV;
    const int sb = sv / 4, st_ = (sv % 4) / 2, sri = sv % 2;
    const int snt = st_ == 0 ? n0 : n1;
    double creg[2][CE], greg = 0.0;
    auto fetch_block = [&](int j) {
        if (a.accumulate && tid < GO) {
            const int step = lo + j * kAdjCB + (tid / 16) * G + sg;
            greg = step < snt ? *gaddr(m + st_ + 2 * step, sb, sri) : 0.0;
        }
#pragma unroll
        for (int e = 0; e < CE; e++) {
            const int el = tid + e * T;
            const int step = lo + j * kAdjCB + el / CW;
            const size_t idx = (size_t)(2 * step + 2) * 4 + el % CW;
            creg[0][e] = step <= n0 ? chd[idx] : 0.0;
            if constexpr (DD) creg[1][e] = step <= n0 ? cld[idx] : 0.0;
        }
    };
    auto stage_block = [&](int slot) {
#pragma unroll
        for (int e = 0; e < CE; e++) {
            cbuf[slot][tid + e * T] = creg[0][e];
            if constexpr (DD) cbuf[slot][kAdjCB * CW + tid + e * T] = creg[1][e];
        }
        if (a.accumulate && tid < GO) gbuf_acc[slot][tid] = greg;
    };
    auto coef = [&](int i, double4 &e4, double4 &o4, double4 &el, double4 &ol) {
        const int j = (i - lo) / kAdjCB, s = (i - lo) % kAdjCB;
        const double4 *cb = reinterpret_cast<const double4 *>(&cbuf[j & 1][s * CW]);
        e4 = cb[0];
        o4 = cb[1];
        if constexpr (DD) {
            const double4 *cbl = reinterpret_cast<const double4 *>(&cbuf[j & 1][kAdjCB * CW + s * CW]);
            el = cbl[0];
            ol = cbl[1];
        }
    };
    fetch_block(0);
    stage_block(0);
    fetch_block(1);
    __syncthreads();

    // reduction role of this thread: output (rg, rv) of a group, slice rs
    const int ro = tid / SL, rs = tid % SL;
    const int rg = ro / NV, rv = ro % NV;               // step in group, component
    const int rb = rv / 4, rt = (rv % 4) / 2, rri = rv % 2;
    const int nt = rt == 0 ? n0 : n1;


    double4 e4, o4, el = {0, 0, 0, 0}, ol = {0, 0, 0, 0};
    coef(lo, e4, o4, el, ol);

    // Steps run in groups of G without a break: the last group may run past
    // n0 (its extra partials are never stored, its coefficients are stale
    // but finite table or LDS values).  A group whose steps all precede the
    // first live chain of the wave (wlo and lo are multiples of kChunk, and
    // G divides kChunk) only writes zero partials; chains join at the first
    // step of a group.
    int buf = 0;
    for (int g0 = lo; g0 < n0; g0 += G, buf ^= 1) {
        double *gbuf = red + (size_t)buf * G * NV * T;
        double *rbuf = gbuf + tid;
        if (g0 + G <= wlo) {
#pragma unroll
            for (int v = 0; v < G * NV; v++) rbuf[v * T] = 0.0;
            coef(g0 + G, e4, o4, el, ol);
        } else {
            if ((g0 % kChunk) == 0 && g0 <= hi) {
#pragma unroll
                for (int r = 0; r < R; r++)
#pragma unroll
                    for (int t = 0; t < 2; t++)
                        if (sid[r][t] == g0) {
                            p0[r][t] = st0[r][t];
                            p1[r][t] = st1[r][t];
                        }
            }
#pragma unroll
            for (int u = 0; u < G; u++) {
                const int i = g0 + u;
                // coefficients of the next step
                double4 e4n, o4n, eln = el, oln = ol;
                coef(i + 1, e4n, o4n, eln, oln);
                // partial sums of this thread's rings: P(i) * ybar^t
                double pe_r[NB], pe_i[NB], po_r[NB], po_i[NB];
#pragma unroll
                for (int b = 0; b < NB; b++) pe_r[b] = pe_i[b] = po_r[b] = po_i[b] = 0.0;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const double pe = p0[r][0].h, po = p0[r][1].h;
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        pe_r[b] = __builtin_fma(pe, yer[r][b], pe_r[b]);
                        pe_i[b] = __builtin_fma(pe, yei[r][b], pe_i[b]);
                        po_r[b] = __builtin_fma(po, yor[r][b], po_r[b]);
                        po_i[b] = __builtin_fma(po, yoi[r][b], po_i[b]);
                    }
                }
                double *rs_ = rbuf + (size_t)u * NV * T;
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    rs_[(4 * b + 0) * T] = pe_r[b];
                    rs_[(4 * b + 1) * T] = pe_i[b];
                    rs_[(4 * b + 2) * T] = po_r[b];
                    rs_[(4 * b + 3) * T] = po_i[b];
                }
                // advance the recurrence
                if constexpr (!DD) {
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        const double pe = p0[r][0].h, po = p0[r][1].h;
                        const double Ae = __builtin_fma(z2h[r], e4.x, e4.y);
                        const double Ao = __builtin_fma(z2h[r], o4.x, o4.y);
                        const double ne = __builtin_fma(Ae, p1[r][0].h, e4.z * pe);
                        const double no = __builtin_fma(Ao, p1[r][1].h, o4.z * po);
                        p0[r][0].h = p1[r][0].h;
                        p1[r][0].h = ne;
                        p0[r][1].h = p1[r][1].h;
                        p1[r][1].h = no;
                    }
                } else {
                    const dd2 Be = {e4.x, el.x}, ABe = {e4.y, el.y}, Ge = {e4.z, el.z};
                    const dd2 Bo = {o4.x, ol.x}, ABo = {o4.y, ol.y}, Go = {o4.z, ol.z};
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        const dd2 z2 = {z2h[r], z2l[r]};
                        const dd2 Ae = dd2_add(dd2_mul(z2, Be), ABe);
                        const dd2 Ao = dd2_add(dd2_mul(z2, Bo), ABo);
                        const dd2 ne = dd2_add(dd2_mul(Ae, p1[r][0]), dd2_mul(Ge, p0[r][0]));
                        const dd2 no = dd2_add(dd2_mul(Ao, p1[r][1]), dd2_mul(Go, p0[r][1]));
                        p0[r][0] = p1[r][0];
                        p1[r][0] = ne;
                        p0[r][1] = p1[r][1];
                        p1[r][1] = no;
                    }
                }
                e4 = e4n;
                o4 = o4n;
                if constexpr (DD) {
                    el = eln;
                    ol = oln;
                }
            }
        }
        __syncthreads();
        // after the first group of block j, block j + 1 goes to LDS (its slot
        // was last read before this barrier) and block j + 2 is fetched
        if ((g0 - lo) % kAdjCB == 0) {
            const int j = (g0 - lo) / kAdjCB;
            stage_block((j + 1) & 1);
            fetch_block(j + 2);
        }
        // reduce the group: slice rs of output (rg, rv) adds partials rs + SL*j
        const double *rp = gbuf + ((size_t)rg * NV + rv) * T + rs;
        double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
        for (int j = 0; j < PS; j += 2) {
            acc0 += rp[SL * j];
            acc1 += rp[SL * (j + 1)];
        }
        double acc = row16_sum(acc0 + acc1);
        const int is = g0 + rg;  // chain step of this output
        if (rs == 0 && is < nt) {
            if (a.accumulate) {
                const int j = (g0 - lo) / kAdjCB, q = ((g0 - lo) % kAdjCB) / G;
                acc += gbuf_acc[j & 1][q * 16 + ro];
            }
            if (m == 0 && rri == 1) acc = 0.0;
            *gaddr(m + rt + 2 * is, rb, rri) = acc;
        }
    }
    // entries before lo are zero
    if (!a.accumulate) {
        for (int e = tid; e < 2 * lo * NB * 2 && e < (L - m + 1) * NB * 2; e += T) {
            const int l = m + e / (NB * 2);
            if (l - m < 2 * lo) *gaddr(l, (e / 2) % NB, e % 2) = 0.0;
        }
    }
}

// FP64 rings on the matrix cores: the sum over rings of each output is a
// product P Y of the Legendre values P (chain step and parity by ring) with
// the unfolded ring phases Y (ring by parity, map and re/im), so it runs as
// MFMA 16x16x4 tiles with the rings as the contraction dimension.
// 512 threads, one ring per lane (8 waves, 512 rings; two workgroups share a
// CU, so that one computes while the other reduces).  Per block of 8
// chain steps every lane writes its ring's 16 values (8 steps x 2 parities)
// to its wave's LDS tile; the wave then multiplies the tile (rows: 8 t + u,
// columns: its 64 rings) by its Y operands (16 per lane, in registers,
// columns 8 t' + c for parity t', map c / 2, re/im c % 2) in 16 MFMAs; rows
// and columns of the same parity are the outputs.  The 8 waves' tiles are
// added through LDS in a fixed order (deterministic).  Chain starts and the
// coefficient blocks follow k_legendre_adj.
typedef double adj_d4 __attribute__((ext_vector_type(4)));
// The value of lane K of each 16-lane row, in every lane of that row.
template <int K>
__device__ __forceinline__ double row_bcast64(double x) {
    return __builtin_amdgcn_mov_dpp(x, 0x150 + K, 0xF, 0xF, false);
}
constexpr int kAdjMfThreads = 512;
constexpr int kAdjMfRow = 65;  // doubles per tile row (64 rings and a pad)

template <int NB>
__global__ __launch_bounds__(kAdjMfThreads) void k_legendre_adj_mf(AdjArgs a) {
    constexpr int T = kAdjMfThreads, SB = 8, CW = 8;
    constexpr int CE = (kAdjCB * CW + T - 1) / T;
    static_assert(2 * NB <= 8 && kChunk == SB && kAdjCB % SB == 0, "tile shape");
    extern __shared__ double tiles[];  // [wave][16 rows][kAdjMfRow]
    __shared__ double cbuf[2][kAdjCB * CW];
    const int m = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int L = a.L;
    const int n0 = (L - m) / 2 + 1;
    const int n1 = (L - m >= 1) ? (L - m - 1) / 2 + 1 : 0;
    const size_t aoff = (size_t)m * (2 * L + 3 - m) / 2;

    __shared__ int s_lo, s_hi;
    if (tid == 0) {
        int lo = kDead, hi = -1;
        for (int gr = a.k0 / kLanes; gr < (a.k1 + kLanes - 1) / kLanes; gr++) {
            lo = min(lo, a.grp_lo[(size_t)m * a.ng + gr]);
            hi = max(hi, a.grp_hi[(size_t)m * a.ng + gr]);
        }
        s_lo = lo;
        s_hi = hi;
    }
    __syncthreads();
    const int lo = s_lo, hi = s_hi;
    auto gaddr = [&](int l, int b, int ri) { return a.g + 2 * ((aoff + l - m) * a.nmaps + a.map0 + b) + ri; };
    if (lo >= n0) {
        if (!a.accumulate)
            for (int e = tid; e < (L - m + 1) * NB * 2; e += T) *gaddr(m + e / (NB * 2), (e / 2) % NB, e % 2) = 0.0;
        return;
    }

    // this lane's ring
    const int k = a.k0 + tid;
    const bool val = k < a.k1 && k < a.n_north;
    const int kk = val ? k : a.k0;
    const double z2 = a.z2_hi[kk];
    int sid[2];
    double p0[2] = {0.0, 0.0}, p1[2] = {0.0, 0.0};
    int wlo = kDead;
#pragma unroll
    for (int t = 0; t < 2; t++) {
        sid[t] = val ? a.start_idx[(size_t)(2 * m + t) * a.np + kk] : kDead;
        wlo = min(wlo, sid[t]);
    }
    wlo = __builtin_amdgcn_readfirstlane(wave_min(wlo));
    // Y operands: MFMA j takes B[l / 16][l % 16] = Y_t'[ring 4 j + l / 16][c]
    double yb[16];
    {
        const int cc = lane & 15, tp = cc >> 3, c = cc & 7, b = c >> 1, ri = c & 1;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const int kr = a.k0 + 64 * wv + 4 * j + (lane >> 4);
            double v = 0.0;
            if (c < 2 * NB && kr < a.k1 && kr < a.n_north) {
                const int ks = a.nrings - 1 - kr;
                const double *yn = reinterpret_cast<const double *>(a.ybar + ((size_t)kr * (L + 1) + m) * a.nmaps +
                                                                    a.map0 + b);
                const double *ys = reinterpret_cast<const double *>(a.ybar + ((size_t)ks * (L + 1) + m) * a.nmaps +
                                                                    a.map0 + b);
                const double vn = yn[ri], vs = ks != kr ? ys[ri] : 0.0;
                v = tp == 0 ? vn + vs : vn - vs;
            }
            yb[j] = v;
        }
    }

    const long long cbase = a.coef_off[m];
    const double *__restrict__ chd = a.coef_hi + 4 * cbase;
    double creg[CE];
    auto fetch_block = [&](int j) {
#pragma unroll
        for (int e = 0; e < CE; e++) {
            const int el = tid + e * T;
            const int step = lo + j * kAdjCB + el / CW;
            const size_t idx = (size_t)(2 * step + 2) * 4 + el % CW;
            creg[e] = (el < kAdjCB * CW && step <= n0) ? chd[idx] : 0.0;
        }
    };
    auto stage_block = [&](int slot) {
#pragma unroll
        for (int e = 0; e < CE; e++)
            if (tid + e * T < kAdjCB * CW) cbuf[slot][tid + e * T] = creg[e];
    };
    fetch_block(0);
    stage_block(0);
    fetch_block(1);
    __syncthreads();

    double *tile = tiles + (size_t)wv * 16 * kAdjMfRow;
    // reduction role (threads 0..127): output row q, column 8 t(q) + c
    const int rq = (tid >> 3) & 15, rc = tid & 7, rt = rq >> 3, ru = rq & 7;
    const int rlane = 16 * (rq & 3) + 8 * rt + rc, rreg = rq >> 2;
    const int nt = rt == 0 ? n0 : n1;
    for (int g0 = lo; g0 < n0; g0 += SB) {
        const int j = (g0 - lo) / kAdjCB, s0 = (g0 - lo) % kAdjCB;
        // the output this thread adds, fetched before the block's work
        const int is = g0 + ru;
        double gold = 0.0;
        if (a.accumulate && tid < 128 && rc < 2 * NB && is < nt) gold = *gaddr(m + rt + 2 * is, rc >> 1, rc & 1);
        adj_d4 acc = {0.0, 0.0, 0.0, 0.0};
        if (g0 + SB > wlo) {
            if ((g0 % kChunk) == 0 && g0 <= hi) {
#pragma unroll
                for (int t = 0; t < 2; t++)
                    if (sid[t] == g0) {  // the chain's two start values, loaded once
                        const size_t row = (size_t)(2 * m + t);
                        p0[t] = a.start_val[(row * 2 + 0) * a.np + kk];
                        p1[t] = a.start_val[(row * 2 + 1) * a.np + kk];
                    }
            }
#pragma unroll
            for (int u = 0; u < SB; u++) {
                // the step's 8 coefficients, one per lane of each 8, reach
                // every lane by DPP broadcasts (one LDS read instead of two
                // 32-byte broadcast reads)
                const double cv = cbuf[j & 1][(s0 + u) * CW + (lane & 7)];
                const double eB = row_bcast64<0>(cv), eAB = row_bcast64<1>(cv), eG = row_bcast64<2>(cv);
                const double oB = row_bcast64<4>(cv), oAB = row_bcast64<5>(cv), oG = row_bcast64<6>(cv);
                tile[u * kAdjMfRow + lane] = p0[0];
                tile[(8 + u) * kAdjMfRow + lane] = p0[1];
                const double ne = __builtin_fma(__builtin_fma(z2, eB, eAB), p1[0], eG * p0[0]);
                const double no = __builtin_fma(__builtin_fma(z2, oB, oAB), p1[1], oG * p0[1]);
                p0[0] = p1[0];
                p1[0] = ne;
                p0[1] = p1[1];
                p1[1] = no;
            }
            // the wave's own tile: its LDS writes and reads complete in order
#pragma unroll
            for (int jj = 0; jj < 16; jj++)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(tile[(lane & 15) * kAdjMfRow + 4 * jj + (lane >> 4)],
                                                           yb[jj], acc, 0, 0, 0);
        }
        // the wave's 16 x 16 sums (element r of lane l: row l / 16 + 4 r,
        // column l % 16) replace its tile, then the waves are added
#pragma unroll
        for (int r = 0; r < 4; r++) tile[r * 64 + lane] = acc[r];
        __syncthreads();
        if ((g0 - lo) % kAdjCB == 0) {  // next coefficient block to LDS, the one after fetched
            stage_block((j + 1) & 1);
            fetch_block(j + 2);
        }
        if (tid < 128 && rc < 2 * NB) {
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < T / 64; w++) sum += tiles[(size_t)w * 16 * kAdjMfRow + rreg * 64 + rlane];
            if (is < nt) {
                sum += gold;
                if (m == 0 && (rc & 1)) sum = 0.0;
                *gaddr(m + rt + 2 * is, rc >> 1, rc & 1) = sum;
            }
        }
        __syncthreads();
    }
    if (!a.accumulate) {
        for (int e = tid; e < 2 * lo * NB * 2 && e < (L - m + 1) * NB * 2; e += T) {
            const int l = m + e / (NB * 2);
            if (l - m < 2 * lo) *gaddr(l, (e / 2) % NB, e % 2) = 0.0;
        }
    }
}

// Defined with the ring kernels: raises a kernel's dynamic LDS limit once
// per (kernel, device).
hipError_t allow_dynamic_lds(const void *fn, int bytes);

template <int T, int R, int NB, bool DD>
static hipError_t launch_adj_cfg(const sht_plan_s *p, AdjArgs a, hipStream_t st) {
    const size_t lds = (size_t)2 * 16 * T * sizeof(double);
    hipError_t ea = allow_dynamic_lds((const void *)k_legendre_adj<T, R, NB, DD>, (int)lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL((k_legendre_adj<T, R, NB, DD>), dim3((unsigned)(p->L + 1)), dim3(T), lds, st, a);
    return hipGetLastError();
}

template <int NB>
static hipError_t launch_adj_mf(const sht_plan_s *p, AdjArgs a, hipStream_t st) {
    const size_t lds = (size_t)(kAdjMfThreads / 64) * 16 * kAdjMfRow * sizeof(double);
    hipError_t ea = allow_dynamic_lds((const void *)k_legendre_adj_mf<NB>, (int)lds);
    if (ea != hipSuccess) return ea;
    hipLaunchKernelGGL((k_legendre_adj_mf<NB>), dim3((unsigned)(p->L + 1)), dim3(kAdjMfThreads), lds, st, a);
    return hipGetLastError();
}

// Double-double rings: 256 threads, one ring each (at most 256 per launch).
template <int NB>
static hipError_t launch_adj_dd(const sht_plan_s *p, AdjArgs a, hipStream_t st) {
    return launch_adj_cfg<256, 1, NB, true>(p, a, st);
}

hipError_t launch_legendre_adjoint(const sht_plan_s *p, int nmaps, const double *ybar, double *g,
                                   hipStream_t stream) {
    AdjArgs a;
    a.z2_hi = p->d_z2_hi;
    a.z2_lo = p->d_z2_lo;
    a.coef_off = p->d_coef_off;
    a.coef_hi = p->d_coef_hi;
    a.coef_lo = p->d_coef_lo;
    a.start_idx = p->d_start_idx;
    a.start_val = p->d_start_val;
    a.start_lo = p->d_start_lo;
    a.grp_lo = p->d_grp_lo;
    a.grp_hi = p->d_grp_hi;
    a.ybar = reinterpret_cast<const double2 *>(ybar);
    a.g = g;
    a.L = p->L;
    a.nrings = p->nrings;
    a.n_north = p->n_north;
    a.np = p->n_north_pad;
    a.n_dd_pad = std::max(p->n_dd_pad, 1);
    a.ng = p->n_north_pad / kLanes;
    a.nmaps = nmaps;
    hipError_t e = hipSuccess;
    const int kdd = std::min(p->n_dd_pad, p->n_north);
    // polar rings (double-double) first, two maps per pass, in chunks of 256
    // rings; the first chunk writes g
    for (int b = 0; b < nmaps && e == hipSuccess;) {
        const int nb = (nmaps - b) >= 2 ? 2 : 1;
        a.map0 = b;
        for (int k0 = 0; k0 < kdd && e == hipSuccess; k0 += 256) {
            a.k0 = k0;
            a.k1 = std::min(kdd, k0 + 256);
            a.accumulate = k0 > 0 ? 1 : 0;
            e = nb == 2 ? launch_adj_dd<2>(p, a, stream) : launch_adj_dd<1>(p, a, stream);
        }
        b += nb;
    }
    // the remaining rings in FP64 on the matrix cores, up to four maps per
    // pass, in chunks of kAdjMfThreads rings, each adding to g
    for (int b = 0; b < nmaps && e == hipSuccess;) {
        const int nb = (nmaps - b) >= 4 ? 4 : (nmaps - b) >= 2 ? 2 : 1;
        a.map0 = b;
        for (int k0 = kdd; k0 < p->n_north && e == hipSuccess; k0 += kAdjMfThreads) {
            a.k0 = k0;
            a.k1 = std::min(p->n_north, k0 + kAdjMfThreads);
            a.accumulate = (kdd > 0 || k0 > kdd) ? 1 : 0;
            e = nb == 4 ? launch_adj_mf<4>(p, a, stream)
                        : nb == 2 ? launch_adj_mf<2>(p, a, stream) : launch_adj_mf<1>(p, a, stream);
        }
        b += nb;
    }
    return e;
}

}  // namespace sht
