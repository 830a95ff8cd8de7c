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
// workgroup owns one order m and every ring it needs: each thread runs the
// two-step recurrence (App. A.2 Eq. A2) for R rings, forms per-step partial
// sums over them, and the workgroup adds the partials of two chain steps at
// a time through LDS in a fixed order (deterministic, no atomics, no
// partial-sum workspace).  Rings nearest the poles run the recurrence in
// double-double arithmetic in their own, smaller workgroups (launched first,
// writing g); the FP64 workgroups then add their share to g in place.
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// T threads, R rings per thread (ring k0 + tid + r*T), NB maps per pass.
// LDS: partials red[2 steps][4*NB components][T].
template <int T, int R, int NB, bool DD>
__global__ __launch_bounds__(T) void k_legendre_adj(AdjArgs a) {
    constexpr int NV = 4 * NB;  // (parity, map, re/im) components per step
    constexpr int NW = T / 64;  // waves
    extern __shared__ double red[];
    const int m = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
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

    auto store = [&](int l, int b, int ri, double v) {
        double *dst = a.g + 2 * ((aoff + l - m) * a.nmaps + a.map0 + b) + ri;
        if (m == 0 && ri == 1) v = 0.0;
        if (a.accumulate) *dst += v;
        else *dst = v;
    };

    if (lo >= n0) {  // every chain of these rings stays below the cutoff
        if (!a.accumulate)
            for (int e = tid; e < (L - m + 1) * NB * 2; e += T) store(m + e / (NB * 2), (e / 2) % NB, e % 2, 0.0);
        return;
    }

    int k[R];
    bool val[R];
    double z2h[R], z2l[R];
    int sid[R][2];
    dd2 st0[R][2], st1[R][2], p0[R][2], p1[R][2];
    double yer[R][NB], yei[R][NB], yor[R][NB], yoi[R][NB];
#pragma unroll
    for (int r = 0; r < R; r++) {
        k[r] = a.k0 + tid + r * T;
        val[r] = k[r] < a.k1 && k[r] < a.n_north;
        const int kk = val[r] ? k[r] : a.k0;
        z2h[r] = a.z2_hi[kk];
        z2l[r] = DD ? a.z2_lo[kk] : 0.0;
#pragma unroll
        for (int t = 0; t < 2; t++) {
            size_t row = (size_t)(2 * m + t);
            sid[r][t] = val[r] ? a.start_idx[row * a.np + kk] : kDead;
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
    const long long cbase = a.coef_off[m];
    const double *__restrict__ ch = a.coef_hi + 4 * cbase;
    const double *__restrict__ cl = a.coef_lo + 4 * cbase;

    for (int c = lo; c < n0; c += kChunk) {
        if (c <= hi) {
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int t = 0; t < 2; t++)
                    if (sid[r][t] == c) {
                        p0[r][t] = st0[r][t];
                        p1[r][t] = st1[r][t];
                    }
        }
        for (int u = 0; u < kChunk; u++) {
            const int i = c + u;
            if (i >= n0) break;
            const int slot = i & 1;
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
            double *rs = red + (size_t)slot * NV * T;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                rs[(4 * b + 0) * T + tid] = pe_r[b];
                rs[(4 * b + 1) * T + tid] = pe_i[b];
                rs[(4 * b + 2) * T + tid] = po_r[b];
                rs[(4 * b + 3) * T + tid] = po_i[b];
            }
            // advance the recurrence
            const double4 *ce4 = reinterpret_cast<const double4 *>(ch) + (2 * i + 2);
            const double4 e4 = ce4[0], o4 = ce4[1];
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
                const double4 *cl4 = reinterpret_cast<const double4 *>(cl) + (2 * i + 2);
                const double4 el = cl4[0], ol = cl4[1];
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
            // every second step (and at the end) the workgroup reduces the
            // partials of the steps held in LDS: wave w sums component w
            if (slot == 1 || i == n0 - 1) {
                __syncthreads();
                const int nsteps = slot + 1;
                for (int o = wave; o < nsteps * NV; o += NW) {
                    const int sl = o / NV, v = o % NV;
                    const double *rv = red + ((size_t)sl * NV + v) * T;
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < T / 64; j++) acc += rv[lane + 64 * j];
                    acc = wave_sum(acc);
                    const int is = i - slot + sl;  // chain index of that step
                    const int b = v / 4, comp = v % 4;
                    const int t = comp / 2, ri = comp % 2;
                    if (lane == 0 && is < (t == 0 ? n0 : n1)) store(m + t + 2 * is, b, ri, acc);
                }
                __syncthreads();
            }
        }
    }
    // chains that never start inside [lo, n0) leave their l untouched only if
    // the whole order is dead, handled above; entries before lo are zero
    if (!a.accumulate) {
        for (int e = tid; e < 2 * lo * NB * 2 && e < (L - m + 1) * NB * 2; e += T) {
            const int l = m + e / (NB * 2);
            if (l - m < 2 * lo) store(l, (e / 2) % NB, e % 2, 0.0);
        }
    }
}

template <int T, int R, int NB, bool DD>
static hipError_t launch_adj_cfg(const sht_plan_s *p, AdjArgs a, hipStream_t st) {
    static bool attr_set = false;
    const size_t lds = (size_t)2 * 4 * NB * T * sizeof(double);
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_legendre_adj<T, R, NB, DD>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
    hipLaunchKernelGGL((k_legendre_adj<T, R, NB, DD>), dim3((unsigned)(p->L + 1)), dim3(T), lds, st, a);
    return hipGetLastError();
}

// FP64 rings: 512 threads, R rings each (R = 1, 2, 4 by the ring count, at
// most 2048 rings per launch).
template <int NB>
static hipError_t launch_adj_fp(const sht_plan_s *p, AdjArgs a, hipStream_t st) {
    const int nr = a.k1 - a.k0;
    if (nr <= 512) return launch_adj_cfg<512, 1, NB, false>(p, a, st);
    if (nr <= 1024) return launch_adj_cfg<512, 2, NB, false>(p, a, st);
    return launch_adj_cfg<512, 4, NB, false>(p, a, st);
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
    for (int b = 0; b < nmaps && e == hipSuccess;) {
        const int nb = (nmaps - b) >= 2 ? 2 : 1;
        a.map0 = b;
        bool wrote = false;
        // polar rings (double-double), in chunks of 256 rings
        for (int k0 = 0; k0 < kdd && e == hipSuccess; k0 += 256) {
            a.k0 = k0;
            a.k1 = std::min(kdd, k0 + 256);
            a.accumulate = wrote ? 1 : 0;
            e = nb == 2 ? launch_adj_dd<2>(p, a, stream) : launch_adj_dd<1>(p, a, stream);
            wrote = true;
        }
        // the remaining rings in FP64, in chunks of up to 2048 rings
        for (int k0 = kdd; k0 < p->n_north && e == hipSuccess; k0 += 2048) {
            a.k0 = k0;
            a.k1 = std::min(p->n_north, k0 + 2048);
            a.accumulate = wrote ? 1 : 0;
            e = nb == 2 ? launch_adj_fp<2>(p, a, stream) : launch_adj_fp<1>(p, a, stream);
            wrote = true;
        }
        b += nb;
    }
    return e;
}

}  // namespace sht
