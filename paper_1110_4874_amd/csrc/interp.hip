// Interpolation form of the Legendre phase (Sec. 3.3 of the Wavemoth paper,
// Eq. 23) for gfx950:
//  1. the phase at the Legendre-root nodes of every (m, parity),
//     q^t_m(z_j) = sum_i a_{m+t+2i} P~_{m+t+2i}^m(z_j), runs in the butterfly
//     residual kernel over the plan's node tasks (per lane a node z_j^2 and
//     the chain's first values above the cutoff), into the workspace;
//  2. k_interp takes every north ring y_k to
//       q^t_m(y_k) = P~_N^m(y_k) sum_j gamma_j q^t_m(z_j) / (y_k^2 - z_j^2),
//     a Cauchy-matrix product on the FP64 matrix cores whose A operand is
//     generated in registers (y^2 - z^2 from double-double parts, so a ring
//     close to a node loses nothing to cancellation), and folds both
//     parities into q rows k and 4 nside - 2 - k (Sec. 2.4, Eqs. 13-14).
// The node phase needs about a third of the brute-force recurrence steps at
// L = 2 nside - 1; the interpolation is a dense product of rings x nodes.
#include "butterfly_common.h"
#include "ddmath.h"

namespace sht {

hipError_t launch_node_phase(const sht_plan_s *p, int nb, BfArgs<double> a, long long npieces, hipStream_t st);

struct IpArgs {
    const long long *__restrict__ node_off;
    const double *__restrict__ x_hi;
    const double *__restrict__ x_lo;
    const double *__restrict__ gam;
    const double *__restrict__ lamN;
    const double *__restrict__ z2_hi;
    const double *__restrict__ z2_lo;
    const double *__restrict__ Q;  // node phases, entries of ES values
    double *__restrict__ q;
    int L, nrings, n_north, np, nmaps, map0, ES, nrb;
};

constexpr int kIpThreads = 256;  // four waves of 16 rings each
constexpr int kIpKS = 4;         // K-steps (4 nodes each) per batch of LDS reads
constexpr int kIpChunk = 256;    // nodes staged in LDS at a time

// 1 / d to a couple of ulps: the hardware estimate refined by two Newton steps
// (each doubles the correct bits), far cheaper than an IEEE division.
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// One workgroup: order m, 64 north rings (16 per wave).  For each parity the
// nodes are staged through LDS in chunks (x_j as hi/lo, and V_j = gamma_j Q_j
// for the 2 NB columns), shared by the four waves; each wave forms the 16 x 4
// Cauchy tile C[ring][j] = 1 / (y^2 - x_j) in registers and accumulates
// S = C V on the matrix cores (columns past 2 NB are zero).  Then
// q(+-y) = P~_N0(y) S_even +- P~_N1(y) S_odd.
template <int NB>
__global__ __launch_bounds__(kIpThreads) void k_interp(IpArgs a) {
    constexpr int NC = 2 * NB;
    __shared__ double sxh[kIpChunk], sxl[kIpChunk];
    __shared__ double sv[kIpChunk * NC];
    // blocks of one order on one XCD (round-robin dispatch over 8 XCDs), so
    // their node phases are shared through that XCD's L2
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int m = 8 * (slot / a.nrb) + xcd, rb = slot % a.nrb;
    if (m > a.L) return;  // uniform over the workgroup
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i16 = lane & 15, k4 = lane >> 4;
    const int ic = min(i16, NC - 1);
    const double cmask = i16 < NC ? 1.0 : 0.0;
    const int k0 = rb * 64 + w * 16;
    const bool active = k0 < a.n_north;
    const int kr = min(k0 + i16, a.np - 1);  // ring of this lane's A-operand row
    const double y2h = a.z2_hi[kr], y2l = a.z2_lo[kr];
    const int nt[2] = {(a.L - m) / 2 + 1, (a.L - m >= 1) ? (a.L - m - 1) / 2 + 1 : 0};
    d4_t acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int t = 0; t < 2; t++) {
        const int n = nt[t];
        const long long base = a.node_off[2 * m + t];
        for (int c0 = 0; c0 < n; c0 += kIpChunk) {
            const int cnt = min(kIpChunk, n - c0);
            __syncthreads();  // the previous chunk has been consumed
            for (int e = tid; e < cnt; e += kIpThreads) {
                sxh[e] = a.x_hi[base + c0 + e];
                sxl[e] = a.x_lo[base + c0 + e];
            }
            for (int e = tid; e < cnt * NC; e += kIpThreads) {
                const int j = e / NC, c = e % NC;
                const long long q = base + c0 + j;
                sv[e] = a.gam[q] * a.Q[(size_t)q * a.ES + c];
            }
            __syncthreads();
            if (!active) continue;
            for (int j0 = 0; j0 < cnt; j0 += 4 * kIpKS) {
                double av[kIpKS], bv[kIpKS];
#pragma unroll
                for (int s = 0; s < kIpKS; s++) {
                    const int j = j0 + 4 * s + k4, jc = min(j, cnt - 1);
                    double d = (y2h - sxh[jc]) + (y2l - sxl[jc]);
                    d = fabs(d) < 1e-200 ? (d < 0 ? -1e-200 : 1e-200) : d;
                    const double valid = j < cnt ? 1.0 : 0.0;
                    av[s] = valid * recip(d);
                    bv[s] = valid * cmask * sv[jc * NC + ic];
                }
#pragma unroll
                for (int s = 0; s < kIpKS; s++) acc[t] = mfma_16x16x4(av[s], bv[s], acc[t]);
            }
        }
    }
    if (!active || i16 >= NC) return;
    const bool odd = nt[1] > 0;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int k = k0 + k4 + 4 * r;  // FP64 accumulator row layout
        if (k >= a.n_north) continue;
        const double le = a.lamN[(size_t)(2 * m) * a.np + k];
        const double lo = odd ? a.lamN[(size_t)(2 * m + 1) * a.np + k] : 0.0;
        const double qe = le * acc[0][r], qo = lo * acc[1][r];
        double vn = qe + qo, vs = qe - qo;
        if (m == 0 && (i16 & 1)) vn = vs = 0.0;  // real field: Im a_l0 is ignored
        const int ks = a.nrings - 1 - k;
        a.q[2 * (((size_t)k * (a.L + 1) + m) * a.nmaps + a.map0) + i16] = vn;
        if (ks != k) a.q[2 * (((size_t)ks * (a.L + 1) + m) * a.nmaps + a.map0) + i16] = vs;
    }
}

// Node phases of the nodes nearest the poles, where an FP64 recurrence
// loses ~l eps / sin(theta): one wave of up to 64 nodes (one per lane) of one
// (m, t), the two-step recurrence of App. A.2 in double-double arithmetic
// (coefficients and z^2 as hi/lo pairs), the sum over the chain in FP64.
struct IpDdArgs {
    const int4 *__restrict__ task;     // [tasks][2]
    const int2 *__restrict__ lane;     // [tasks*64]
    const double4 *__restrict__ val;   // [tasks*64] P0 hi, lo, P1 hi, lo
    const double *__restrict__ x_hi;
    const double *__restrict__ x_lo;
    const long long *__restrict__ coef_off;
    const double *__restrict__ coef_hi;
    const double *__restrict__ coef_lo;
    const double *__restrict__ alm;
    double *__restrict__ Q;
    int L, nmaps, map0, ES;
};

template <int NB>
__global__ __launch_bounds__(64) void k_node_dd(IpDdArgs a) {
    constexpr int NC = 2 * NB;
    const int lane = threadIdx.x;
    const int4 h = a.task[2 * blockIdx.x], h2 = a.task[2 * blockIdx.x + 1];
    const int t = __builtin_amdgcn_readfirstlane(h.x), m = __builtin_amdgcn_readfirstlane(h.y);
    const int n = __builtin_amdgcn_readfirstlane(h.z), nl = __builtin_amdgcn_readfirstlane(h.w);
    const int outb = __builtin_amdgcn_readfirstlane(h2.x), lane0 = __builtin_amdgcn_readfirstlane(h2.y);
    const int imin = __builtin_amdgcn_readfirstlane(h2.z);
    const int2 ln = a.lane[(size_t)lane0 + lane];
    const double4 sv = a.val[(size_t)lane0 + lane];
    const int i0 = ln.y;
    const dd z2 = {a.x_hi[ln.x], a.x_lo[ln.x]};
    dd P0 = {0.0, 0.0}, P1 = {0.0, 0.0};
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) acc[c] = 0.0;
    c_double *ch = (c_double *)(a.coef_hi + 4 * a.coef_off[m]);
    c_double *cl = (c_double *)(a.coef_lo + 4 * a.coef_off[m]);
    const size_t aoff = (size_t)m * (2 * a.L + 3 - m) / 2;
    c_double *ap = (c_double *)(a.alm + 2 * ((aoff + t) * a.nmaps + a.map0));
    const size_t astride = 4 * (size_t)a.nmaps;  // doubles between chain rows i and i + 1
    for (int i = imin; i < n; i++) {
        if (i == i0) {
            P0 = {sv.x, sv.y};
            P1 = {sv.z, sv.w};
        }
#pragma unroll
        for (int c = 0; c < NC; c++) acc[c] = __builtin_fma(P0.h, ap[(size_t)i * astride + c], acc[c]);
        const int e = 4 * (t + 2 * i + 2);
        const dd B = {ch[e], cl[e]}, AB = {ch[e + 1], cl[e + 1]}, G = {ch[e + 2], cl[e + 2]};
        const dd A = dd_add(dd_mul(z2, B), AB);
        const dd P2 = dd_add(dd_mul(A, P1), dd_mul(G, P0));
        P0 = P1;
        P1 = P2;
    }
    if (lane < nl) {
        double *dst = a.Q + ((size_t)outb + lane) * a.ES;
#pragma unroll
        for (int c = 0; c < NC; c++) dst[c] = acc[c];
    }
}

// Rings evaluated at the ring itself (closer to a node than the nodes'
// precision allows for): both parities' values, from their node slots, are
// folded into q rows k and 4 nside - 2 - k over what k_interp wrote.  One
// thread per (patch, column).
struct IpPatchArgs {
    const int4 *__restrict__ patch;  // {m, ring, slot of t = 0, slot of t = 1}
    const double *__restrict__ Q;
    double *__restrict__ q;
    int L, nrings, nmaps, map0, ES, npatch;
};

template <int NB>
__global__ __launch_bounds__(256) void k_interp_patch(IpPatchArgs a) {
    constexpr int NC = 2 * NB;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long long)a.npatch * NC) return;
    const int pi = (int)(e / NC), c = (int)(e % NC);
    const int4 pt = a.patch[pi];
    const int m = pt.x, k = pt.y;
    const double qe = pt.z >= 0 ? a.Q[(size_t)pt.z * a.ES + c] : 0.0;
    const double qo = pt.w >= 0 ? a.Q[(size_t)pt.w * a.ES + c] : 0.0;
    double vn = qe + qo, vs = qe - qo;
    if (m == 0 && (c & 1)) vn = vs = 0.0;  // real field: Im a_l0 is ignored
    const int ks = a.nrings - 1 - k;
    a.q[2 * (((size_t)k * (a.L + 1) + m) * a.nmaps + a.map0) + c] = vn;
    if (ks != k) a.q[2 * (((size_t)ks * (a.L + 1) + m) * a.nmaps + a.map0) + c] = vs;
}

size_t interp_scratch_bytes(const sht_plan_s *p, int nmaps) {
    const int nb = nmaps >= 4 ? 4 : nmaps >= 2 ? 2 : 1;
    return (size_t)p->ip.nodes * 2 * nb * sizeof(double);
}

template <int NB>
static hipError_t launch_interp_nb(const sht_plan_s *p, IpArgs ia, hipStream_t st) {
    const long long morders = (p->L + 1 + 7) / 8 * 8;
    const long long grid = morders * ia.nrb;
    hipLaunchKernelGGL((k_interp<NB>), dim3((unsigned)grid), dim3(kIpThreads), 0, st, ia);
    return hipGetLastError();
}

hipError_t launch_interp(const sht_plan_s *p, int nmaps, const double *alm, double *q, void *scratch,
                         hipStream_t stream) {
    const InterpPlan &ip = p->ip;
    BfArgs<double> a = bf_args<double>(p, nmaps, nullptr, (double *)scratch);
    a.res_sub = reinterpret_cast<const int4 *>(p->d_ip_sub);
    a.res_lane = reinterpret_cast<const int2 *>(p->d_ip_lane);
    a.res_val = reinterpret_cast<const double2 *>(p->d_ip_val);
    a.z2 = p->d_ip_x_hi;
    a.alm = reinterpret_cast<const double2 *>(alm);
    const long long npieces = (long long)ip.sub.size() / 8;
    IpArgs ia;
    ia.node_off = p->d_ip_node_off;
    ia.x_hi = p->d_ip_x_hi;
    ia.x_lo = p->d_ip_x_lo;
    ia.gam = p->d_ip_gam;
    ia.lamN = p->d_ip_lamN;
    ia.z2_hi = p->d_z2_hi;
    ia.z2_lo = p->d_z2_lo;
    ia.Q = (const double *)scratch;
    ia.q = q;
    ia.L = p->L;
    ia.nrings = p->nrings;
    ia.n_north = p->n_north;
    ia.np = p->n_north_pad;
    ia.nmaps = nmaps;
    ia.nrb = (p->n_north + 63) / 64;
    IpDdArgs da;
    da.task = reinterpret_cast<const int4 *>(p->d_ip_dd_task);
    da.lane = reinterpret_cast<const int2 *>(p->d_ip_dd_lane);
    da.val = reinterpret_cast<const double4 *>(p->d_ip_dd_val);
    da.x_hi = p->d_ip_x_hi;
    da.x_lo = p->d_ip_x_lo;
    da.coef_off = p->d_coef_off;
    da.coef_hi = p->d_coef_hi;
    da.coef_lo = p->d_coef_lo;
    da.alm = alm;
    da.Q = (double *)scratch;
    da.L = p->L;
    da.nmaps = nmaps;
    const long long ndd = (long long)ip.dd_task.size() / 8;
    IpPatchArgs pa;
    pa.patch = reinterpret_cast<const int4 *>(p->d_ip_patch);
    pa.Q = (const double *)scratch;
    pa.q = q;
    pa.L = p->L;
    pa.nrings = p->nrings;
    pa.nmaps = nmaps;
    pa.npatch = (int)(ip.patch.size() / 4);
    hipError_t e = hipSuccess;
    for (int b = 0; b < nmaps && e == hipSuccess;) {
        const int left = nmaps - b, nb = left >= 4 ? 4 : left >= 2 ? 2 : 1;
        a.map0 = b;
        a.ES = 2 * nb;
        a.G = 1;
        ia.map0 = b;
        ia.ES = 2 * nb;
        da.map0 = b;
        da.ES = 2 * nb;
        e = launch_node_phase(p, nb, a, npieces, stream);
        if (e != hipSuccess) break;
        if (ndd > 0) {
            switch (nb) {
                case 4: hipLaunchKernelGGL((k_node_dd<4>), dim3((unsigned)ndd), dim3(64), 0, stream, da); break;
                case 2: hipLaunchKernelGGL((k_node_dd<2>), dim3((unsigned)ndd), dim3(64), 0, stream, da); break;
                default: hipLaunchKernelGGL((k_node_dd<1>), dim3((unsigned)ndd), dim3(64), 0, stream, da); break;
            }
            if ((e = hipGetLastError()) != hipSuccess) break;
        }
        switch (nb) {
            case 4: e = launch_interp_nb<4>(p, ia, stream); break;
            case 2: e = launch_interp_nb<2>(p, ia, stream); break;
            default: e = launch_interp_nb<1>(p, ia, stream); break;
        }
        if (e != hipSuccess) break;
        if (pa.npatch > 0) {
            pa.map0 = b;
            pa.ES = 2 * nb;
            const dim3 g((unsigned)(((long long)pa.npatch * 2 * nb + 255) / 256));
            switch (nb) {
                case 4: hipLaunchKernelGGL((k_interp_patch<4>), g, dim3(256), 0, stream, pa); break;
                case 2: hipLaunchKernelGGL((k_interp_patch<2>), g, dim3(256), 0, stream, pa); break;
                default: hipLaunchKernelGGL((k_interp_patch<1>), g, dim3(256), 0, stream, pa); break;
            }
            e = hipGetLastError();
        }
        b += nb;
    }
    return e;
}

}  // namespace sht
