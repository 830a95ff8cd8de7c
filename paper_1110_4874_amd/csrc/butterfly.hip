// Butterfly-compressed Legendre phase for gfx950 (Sec. 4.2 and App. A.1 of
// the Wavemoth paper): q^t_m = Lambda^T a^t applied as
//   a^T Lambda = (a^T R) S_d P_{d-1} ... P_1 S_1,
// followed by the even/odd fold of Sec. 2.4 (Eqs. 13-14).
//
// One workgroup owns one order m (both parities) at a time, taking orders
// in the plan's decreasing-work order with a grid stride, and runs:
//  1. the residual R: one thread per (leaf, skeleton ring) lane regenerates
//     Legendre values with the two-step recurrence (App. A.2, Eq. A2) over
//     the leaf's rows from two stored values and accumulates
//     v = sum_l a_lm P~_l^m(z) for every map;
//  2. the levels, deepest first: one thread per output column c of a pair
//     node (two sibling row blocks sharing the column set C) computes
//     u_c = sum_{child} (identity: v[s] | dense: sum_s T[s][d] v[s]), which
//     is the input vector of the next level (level 1 yields q^t per ring);
//     the dense interpolation blocks T are streamed from HBM once per call;
//  3. the fold into q rows k and 4 nside - k (the equator once).
// Vectors live in a per-workgroup slot of device scratch (L2/MALL resident),
// with __syncthreads() between phases.
#include "internal.h"

namespace sht {

template <typename S>
struct BfArgs {
    const int *__restrict__ order;
    const long long *__restrict__ res_off;
    const int4 *__restrict__ res_rec;
    const double2 *__restrict__ res_val;
    const long long *__restrict__ unit_off;
    const int *__restrict__ unit_node;
    const int *__restrict__ code;
    const int *__restrict__ node_i;
    const long long *__restrict__ node_T;
    const S *__restrict__ T;
    const double *__restrict__ z2;
    const long long *__restrict__ coef_off;
    const double *__restrict__ coef;
    const double2 *__restrict__ alm;
    double2 *__restrict__ q;
    S *__restrict__ scratch;
    int L, K, nrings, nmaps, map0, nitems;
    long long slot_entries;
};

constexpr int kBfThreads = 256;

__device__ __forceinline__ double fma_s(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_s(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int NB, typename S>
__global__ __launch_bounds__(kBfThreads) void k_butterfly(BfArgs<S> a) {
    constexpr int NC = 2 * NB;  // components per vector entry
    const int tid = threadIdx.x;
    S *__restrict__ slot = a.scratch + (size_t)blockIdx.x * a.slot_entries * NC;
    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        const int m = a.order[item];
        const size_t aoff = (size_t)m * (2 * a.L + 3 - m) / 2;
        const double4 *__restrict__ cf = reinterpret_cast<const double4 *>(a.coef) + a.coef_off[m];

        // 1. residual lanes
        const long long r0 = a.res_off[m], r1 = a.res_off[m + 1];
        for (long long r = r0 + tid; r < r1; r += kBfThreads) {
            const int4 rec = a.res_rec[r];
            const double2 sv = a.res_val[r];
            const int t = rec.w & 1;
            const long long out = rec.w >> 1;
            const double z2 = a.z2[rec.x];
            double P0 = sv.x, P1 = sv.y;
            double acc[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) acc[c] = 0.0;
            const double2 *ap = a.alm + (aoff + t) * a.nmaps + a.map0;
            for (int i = rec.y; i < rec.z; i++) {
                const double2 *ai = ap + (size_t)2 * i * a.nmaps;
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    const double2 v = ai[b];
                    acc[2 * b] = __builtin_fma(P0, v.x, acc[2 * b]);
                    acc[2 * b + 1] = __builtin_fma(P0, v.y, acc[2 * b + 1]);
                }
                const double4 e = cf[t + 2 * i + 2];
                const double P2 = __builtin_fma(__builtin_fma(z2, e.x, e.y), P1, e.z * P0);
                P0 = P1;
                P1 = P2;
            }
            S *dst = slot + out * NC;
#pragma unroll
            for (int c = 0; c < NC; c++) dst[c] = (S)acc[c];
        }
        __syncthreads();

        // 2. levels, deepest first
        const long long *uo = a.unit_off + (size_t)m * (kBfMaxLv + 1);
        for (int lq = 0; lq < kBfMaxLv; lq++) {
            const long long u0 = uo[lq], u1 = uo[lq + 1];
            if (u0 == u1) continue;
            for (long long u = u0 + tid; u < u1; u += kBfThreads) {
                const int node = a.unit_node[u];
                const int *ni = a.node_i + (size_t)node * kBfNodeInts;
                const int code = a.code[u];
                const int c = (int)(u - ni[7]);
                S acc[NC];
#pragma unroll
                for (int q = 0; q < NC; q++) acc[q] = (S)0;
#pragma unroll
                for (int ch = 0; ch < 2; ch++) {
                    const int cd = (int)(short)(ch == 0 ? (code & 0xffff) : ((unsigned)code >> 16));
                    const S *v = slot + (size_t)ni[ch] * NC;
                    if (cd >= 0) {
#pragma unroll
                        for (int q = 0; q < NC; q++) acc[q] += v[(size_t)cd * NC + q];
                    } else {
                        const int d = -1 - cd, kk = ni[2 + ch], nd = ni[4 + ch];
                        const S *__restrict__ Tp = a.T + a.node_T[2 * node + ch] + d;
                        for (int s = 0; s < kk; s++) {
                            const S w = Tp[(size_t)s * nd];
#pragma unroll
                            for (int q = 0; q < NC; q++) acc[q] = fma_s(w, v[(size_t)s * NC + q], acc[q]);
                        }
                    }
                }
                S *dst = slot + ((size_t)ni[6] + c) * NC;
#pragma unroll
                for (int q = 0; q < NC; q++) dst[q] = acc[q];
            }
            __syncthreads();
        }

        // 3. fold q^even, q^odd into the north ring and its mirror
        const int K = a.K;
        for (int e = tid; e < K * NB; e += kBfThreads) {
            const int k = e / NB, b = e % NB;
            const S *qe = slot + (size_t)k * NC + 2 * b;
            const S *qo = slot + (size_t)(K + k) * NC + 2 * b;
            double er = (double)qe[0], ei = (double)qe[1], orr = (double)qo[0], oi = (double)qo[1];
            if (m == 0) ei = oi = 0.0;
            a.q[((size_t)m * a.nrings + k) * a.nmaps + a.map0 + b] = make_double2(er + orr, ei + oi);
            const int ks = a.nrings - 1 - k;
            if (ks != k) a.q[((size_t)m * a.nrings + ks) * a.nmaps + a.map0 + b] = make_double2(er - orr, ei - oi);
        }
        __syncthreads();
    }
}

int bf_slots(const sht_plan_s *p) { return std::min(p->L + 1, 1024); }

size_t bf_scratch_bytes(const sht_plan_s *p, int nmaps, int fp32) {
    const int nb = nmaps >= 8 ? 8 : nmaps >= 4 ? 4 : nmaps >= 2 ? 2 : 1;
    return (size_t)bf_slots(p) * (size_t)p->bf.slot_entries * 2 * nb * (fp32 ? sizeof(float) : sizeof(double));
}

template <int NB, typename S>
static hipError_t launch_bf_nb(const sht_plan_s *p, BfArgs<S> a, hipStream_t st) {
    hipLaunchKernelGGL((k_butterfly<NB, S>), dim3((unsigned)bf_slots(p)), dim3(kBfThreads), 0, st, a);
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_bf(const sht_plan_s *p, int nmaps, const double *alm, double *q, S *scratch,
                            const S *T, hipStream_t st) {
    BfArgs<S> a;
    a.order = p->d_bf_order;
    a.res_off = p->d_bf_res_off;
    a.res_rec = reinterpret_cast<const int4 *>(p->d_bf_res_rec);
    a.res_val = reinterpret_cast<const double2 *>(p->d_bf_res_val);
    a.unit_off = p->d_bf_unit_off;
    a.unit_node = p->d_bf_unit_node;
    a.code = p->d_bf_code;
    a.node_i = p->d_bf_node_i;
    a.node_T = p->d_bf_node_T;
    a.T = T;
    a.z2 = p->d_z2_hi;
    a.coef_off = p->d_coef_off;
    a.coef = p->d_coef_hi;
    a.alm = reinterpret_cast<const double2 *>(alm);
    a.q = reinterpret_cast<double2 *>(q);
    a.scratch = scratch;
    a.L = p->L;
    a.K = p->bf.K;
    a.nrings = p->nrings;
    a.nmaps = nmaps;
    a.nitems = p->L + 1;
    a.slot_entries = p->bf.slot_entries;
    hipError_t e = hipSuccess;
    for (int b = 0; b < nmaps && e == hipSuccess;) {
        const int rem = nmaps - b;
        a.map0 = b;
        if (rem >= 8) {
            e = launch_bf_nb<8, S>(p, a, st);
            b += 8;
        } else if (rem >= 4) {
            e = launch_bf_nb<4, S>(p, a, st);
            b += 4;
        } else if (rem >= 2) {
            e = launch_bf_nb<2, S>(p, a, st);
            b += 2;
        } else {
            e = launch_bf_nb<1, S>(p, a, st);
            b += 1;
        }
    }
    return e;
}

hipError_t launch_butterfly(const sht_plan_s *p, int nmaps, const double *alm, double *q, void *scratch,
                            int fp32, hipStream_t stream) {
    if (fp32) return launch_bf<float>(p, nmaps, alm, q, (float *)scratch, p->d_bf_T32, stream);
    return launch_bf<double>(p, nmaps, alm, q, (double *)scratch, p->d_bf_T, stream);
}

}  // namespace sht
