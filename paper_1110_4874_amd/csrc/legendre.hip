// Brute-force Legendre phase (Wavemoth paper, Sec. 2.4 Eqs. 12-14 and
// App. A.2 Eqs. A1-A2), for gfx950.
//
//   q_m(+-z_k) = q^even_m(z_k) +- q^odd_m(z_k),
//   q^t_m(z)   = sum_i P~_{m+t+2i}^m(z) a_{m+t+2i, m}
//
// One wavefront handles one order m and a block of 64 x kRingsPerLane
// north rings; every lane owns kRingsPerLane rings and runs both parity
// chains of the two-step recurrence for them.  The recurrence coefficients
// and the a_lm of the current l are the same for every lane, so they are
// read as wave-uniform (scalar) loads and used straight from SGPRs; P~ never
// leaves VGPRs (the GPU form of the paper's register-resident SSE kernel).
// The even/odd fold of Eqs. 13-14 is fused into the store: each lane writes
// ring k and its mirror 4N-2-k.
//
// Chains start at the plan's precomputed values (first l above the cutoff,
// rounded down to a multiple of kChunk chain steps), so a lane joins the
// wave-uniform l loop only at chunk boundaries.  Ring blocks nearest the
// poles, where a z-based FP64 recurrence loses ~l eps / sin(theta), run the
// same recurrence in double-double arithmetic.
#include "internal.h"

namespace sht {

struct LegArgs {
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
    const double *__restrict__ alm;
    double *__restrict__ q;
    int L, nrings, n_north, np, n_dd_pad, ng;
    int nmaps, map0;  // map stride of alm/q and first map of this pass
    int rb0, nrb;     // ring blocks covered by this launch
};

// ---- double-double helpers (error-free transformations) --------------
struct dd {
    double h, l;
};

#pragma clang fp contract(off)
__device__ __forceinline__ dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
    double p = a.h * b.h;
    double e = __builtin_fma(a.h, b.h, -p);
    e = __builtin_fma(a.h, b.l, e);
    e = __builtin_fma(a.l, b.h, e);
    return fast_two_sum(p, e);
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    dd s = two_sum(a.h, b.h);
    double e = s.l + (a.l + b.l);
    return fast_two_sum(s.h, e);
}
#pragma clang fp contract(on)

template <int NB, bool DD>
__global__ __launch_bounds__(64) void k_legendre(LegArgs a) {
    constexpr int R = kRingsPerLane;
    const int blk = blockIdx.x;
    const int m = blk / a.nrb;
    const int rb = a.rb0 + blk % a.nrb;
    const int lane = threadIdx.x;
    const int L = a.L;

    int k[R];
#pragma unroll
    for (int r = 0; r < R; r++) k[r] = rb * kBlockRings + r * kLanes + lane;

    // wave-uniform chain range of this block
    int lo = kDead, hi = -1;
#pragma unroll
    for (int r = 0; r < R; r++) {
        int g = rb * R + r;
        lo = min(lo, a.grp_lo[(size_t)m * a.ng + g]);
        hi = max(hi, a.grp_hi[(size_t)m * a.ng + g]);
    }
    const int n0 = (L - m) / 2 + 1;                    // even chain length
    const int n1 = (L - m >= 1) ? (L - m - 1) / 2 + 1 : 0;  // odd chain length

    double ae_r[NB], ae_i[NB], ao_r[NB], ao_i[NB];
    double accE_r[R][NB], accE_i[R][NB], accO_r[R][NB], accO_i[R][NB];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int b = 0; b < NB; b++) accE_r[r][b] = accE_i[r][b] = accO_r[r][b] = accO_i[r][b] = 0.0;

    if (lo < n0) {
        double z2h[R], z2l[R];
        int sid[R][2];
        dd st0[R][2], st1[R][2], p0[R][2], p1[R][2];
#pragma unroll
        for (int r = 0; r < R; r++) {
            z2h[r] = a.z2_hi[k[r]];
            z2l[r] = DD ? a.z2_lo[k[r]] : 0.0;
#pragma unroll
            for (int t = 0; t < 2; t++) {
                size_t row = (size_t)(2 * m + t);
                sid[r][t] = a.start_idx[row * a.np + k[r]];
                st0[r][t].h = a.start_val[(row * 2 + 0) * a.np + k[r]];
                st1[r][t].h = a.start_val[(row * 2 + 1) * a.np + k[r]];
                st0[r][t].l = DD ? a.start_lo[(row * 2 + 0) * a.n_dd_pad + k[r]] : 0.0;
                st1[r][t].l = DD ? a.start_lo[(row * 2 + 1) * a.n_dd_pad + k[r]] : 0.0;
                p0[r][t] = {0.0, 0.0};
                p1[r][t] = {0.0, 0.0};
            }
        }
        const long long cbase = a.coef_off[m];
        const double *__restrict__ ch = a.coef_hi + 4 * cbase;
        const double *__restrict__ cl = a.coef_lo + 4 * cbase;
        const size_t aoff = (size_t)m * (2 * L + 3 - m) / 2;
        const double *__restrict__ al = a.alm + 2 * (aoff * a.nmaps + a.map0);
        const int astride = 2 * a.nmaps;  // doubles between consecutive l

        auto inject = [&](int c) {
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int t = 0; t < 2; t++)
                    if (sid[r][t] == c) {
                        p0[r][t] = st0[r][t];
                        p1[r][t] = st1[r][t];
                    }
        };

        // one chain step i for both parities: accumulate P(i) a_l, advance
        auto step = [&](int i, bool odd_ok) {
            const double *ce = ch + 4 * (2 * i + 2);  // l = m + 2i + 2 (even), next entry odd
            const double be = ce[0], abe = ce[1], ge = ce[2];
            const double bo = ce[4], abo = ce[5], go = ce[6];
            const double *ape = al + (size_t)(2 * i) * astride;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                ae_r[b] = ape[2 * b];
                ae_i[b] = ape[2 * b + 1];
                ao_r[b] = odd_ok ? ape[astride + 2 * b] : 0.0;
                ao_i[b] = odd_ok ? ape[astride + 2 * b + 1] : 0.0;
            }
            if constexpr (!DD) {
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const double pe = p0[r][0].h, po = p0[r][1].h;
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        accE_r[r][b] = __builtin_fma(pe, ae_r[b], accE_r[r][b]);
                        accE_i[r][b] = __builtin_fma(pe, ae_i[b], accE_i[r][b]);
                        accO_r[r][b] = __builtin_fma(po, ao_r[b], accO_r[r][b]);
                        accO_i[r][b] = __builtin_fma(po, ao_i[b], accO_i[r][b]);
                    }
                    const double Ae = __builtin_fma(z2h[r], be, abe);
                    const double Ao = __builtin_fma(z2h[r], bo, abo);
                    const double ne = __builtin_fma(Ae, p1[r][0].h, ge * pe);
                    const double no = __builtin_fma(Ao, p1[r][1].h, go * po);
                    p0[r][0].h = p1[r][0].h;
                    p1[r][0].h = ne;
                    p0[r][1].h = p1[r][1].h;
                    p1[r][1].h = no;
                }
            } else {
                const double *cle = cl + 4 * (2 * i + 2);
                const dd Be = {be, cle[0]}, ABe = {abe, cle[1]}, Ge = {ge, cle[2]};
                const dd Bo = {bo, cle[4]}, ABo = {abo, cle[5]}, Go = {go, cle[6]};
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const double pe = p0[r][0].h, po = p0[r][1].h;
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        accE_r[r][b] = __builtin_fma(pe, ae_r[b], accE_r[r][b]);
                        accE_i[r][b] = __builtin_fma(pe, ae_i[b], accE_i[r][b]);
                        accO_r[r][b] = __builtin_fma(po, ao_r[b], accO_r[r][b]);
                        accO_i[r][b] = __builtin_fma(po, ao_i[b], accO_i[r][b]);
                    }
                    const dd z2 = {z2h[r], z2l[r]};
                    const dd Ae = dd_add(dd_mul(z2, Be), ABe);
                    const dd Ao = dd_add(dd_mul(z2, Bo), ABo);
                    const dd ne = dd_add(dd_mul(Ae, p1[r][0]), dd_mul(Ge, p0[r][0]));
                    const dd no = dd_add(dd_mul(Ao, p1[r][1]), dd_mul(Go, p0[r][1]));
                    p0[r][0] = p1[r][0];
                    p1[r][0] = ne;
                    p0[r][1] = p1[r][1];
                    p1[r][1] = no;
                }
            }
        };

        // chunks where both chains are inside l <= L
        const int c_full = (n1 / kChunk) * kChunk;
        int c = lo;
        for (; c < c_full; c += kChunk) {
            if (c <= hi) inject(c);
#pragma unroll
            for (int u = 0; u < kChunk; u++) step(c + u, true);
        }
        // tail: the odd chain may end first
        for (; c < n0; c += kChunk) {
            if (c <= hi) inject(c);
            for (int u = 0; u < kChunk; u++) {
                int i = c + u;
                if (i >= n0) break;
                step(i, i < n1);
            }
        }
    }

    // fused even/odd fold and store (Eqs. 13-14)
#pragma unroll
    for (int r = 0; r < R; r++) {
        if (k[r] >= a.n_north) continue;
        const int kn = k[r], ks = a.nrings - 1 - k[r];
        double *qn = a.q + 2 * (((size_t)m * a.nrings + kn) * a.nmaps + a.map0);
        double *qs = a.q + 2 * (((size_t)m * a.nrings + ks) * a.nmaps + a.map0);
#pragma unroll
        for (int b = 0; b < NB; b++) {
            double nr = accE_r[r][b] + accO_r[r][b], ni = accE_i[r][b] + accO_i[r][b];
            double sr = accE_r[r][b] - accO_r[r][b], si = accE_i[r][b] - accO_i[r][b];
            if (m == 0) ni = si = 0.0;  // real field: Im a_l0 is ignored
            *reinterpret_cast<double2 *>(qn + 2 * b) = make_double2(nr, ni);
            if (ks != kn) *reinterpret_cast<double2 *>(qs + 2 * b) = make_double2(sr, si);
        }
    }
}

template <int NB>
static hipError_t launch_nb(const sht_plan_s *p, LegArgs a, hipStream_t st) {
    const int nblocks = p->n_north_pad / kBlockRings;
    // compensated blocks first (they sit nearest the poles), then the rest
    if (p->n_dd_blocks > 0) {
        a.rb0 = 0;
        a.nrb = p->n_dd_blocks;
        hipLaunchKernelGGL((k_legendre<NB, true>), dim3((unsigned)((p->L + 1) * a.nrb)), dim3(kLanes), 0,
                           st, a);
    }
    if (nblocks > p->n_dd_blocks) {
        a.rb0 = p->n_dd_blocks;
        a.nrb = nblocks - p->n_dd_blocks;
        hipLaunchKernelGGL((k_legendre<NB, false>), dim3((unsigned)((p->L + 1) * a.nrb)), dim3(kLanes), 0,
                           st, a);
    }
    return hipGetLastError();
}

hipError_t launch_legendre(const sht_plan_s *p, int nmaps, const double *alm, double *q,
                           hipStream_t stream) {
    LegArgs a;
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
    a.alm = alm;
    a.q = q;
    a.L = p->L;
    a.nrings = p->nrings;
    a.n_north = p->n_north;
    a.np = p->n_north_pad;
    a.n_dd_pad = std::max(p->n_dd_pad, 1);
    a.ng = p->n_north_pad / kLanes;
    a.nmaps = nmaps;
    hipError_t e = hipSuccess;
    // maps in passes of 4, then 2, then 1
    int b = 0;
    while (b < nmaps && e == hipSuccess) {
        a.map0 = b;
        int left = nmaps - b;
        if (left >= 4) {
            e = launch_nb<4>(p, a, stream);
            b += 4;
        } else if (left >= 2) {
            e = launch_nb<2>(p, a, stream);
            b += 2;
        } else {
            e = launch_nb<1>(p, a, stream);
            b += 1;
        }
    }
    return e;
}

}  // namespace sht
