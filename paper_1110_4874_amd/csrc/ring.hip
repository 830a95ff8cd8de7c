// Ring stage of synthesis (Wavemoth paper, Sec. 2.3 Eqs. 8-11), for gfx950.
//
// For ring k with J pixels at phi_j = pi (2j + s) / J:
//   f_j = sum_{m=-L}^{L} q_m e^{i m phi_j},   q_{-m} = conj(q_m)
//       = sum_{b=0}^{J-1} X_b e^{2 pi i b j / J},
//   X_b = sum_{m = b mod J} q_m e^{i pi m s / J}        (phase shift + wrap)
// X is Hermitian, so f is the real backward DFT of X; it is computed as a
// complex DFT of half length n = J/2 (even and odd pixels in the real and
// imaginary parts) after the usual pre-twiddle.
//
// One workgroup handles one (ring, map).  Bin b gathers the m in its two
// residue classes m = b + jJ and m = jJ - b; all of them share the phase
// e^{i pi b s/J} up to the sign (-1)^{js}, so each bin needs one sincospi.
// Small rings split the m range over thread groups and reduce in a fixed
// order (deterministic, no atomics).  The half-length DFT runs in LDS:
// radix-2 in place when n is a power of two (input written bit-reversed),
// otherwise Bluestein's chirp convolution with a power-of-two M >= 2n-1
// whose chirp spectrum is a plan table.  Workgroups are ordered so that the
// 8 (ring, map) pairs whose q entries share a 128-byte line run back to back
// on the same XCD (dispatch is round-robin over the 8 XCDs).
#include "internal.h"

namespace sht {

struct RingArgs {
    const int *__restrict__ rings;
    int count;
    const int *__restrict__ ring_J;
    const int *__restrict__ ring_s;
    const int *__restrict__ ring_M;
    const long long *__restrict__ ring_off;
    const long long *__restrict__ ring_bs_off;
    const double2 *__restrict__ tw;
    int tw_log;
    const double2 *__restrict__ bs_table;
    const double2 *__restrict__ q;
    double *__restrict__ map;
    int L, nrings, nmaps;
    long long npix;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 expipi(double x) {  // e^{i pi x}
    double s, c;
    sincospi(x, &s, &c);
    return make_double2(c, s);
}
__device__ __forceinline__ int ilog2_dev(int n) { return 31 - __clz(n); }
__device__ __forceinline__ int bitrev(int k, int lg) { return lg == 0 ? 0 : (int)(__brev((unsigned)k) >> (32 - lg)); }

// Workgroup -> work item, grouping 8 consecutive items on one XCD.
__device__ __forceinline__ int xcd_item(int wg) { return (wg & ~63) + ((wg & 7) << 3) + ((wg >> 3) & 7); }

// In-place radix-2 decimation-in-time DFT of size 2^lg, bit-reversed input,
// natural output, sign +1 (backward): a_p <- sum_k a_k e^{+2 pi i k p / n}.
__device__ void fft_dit_inv(double2 *a, int lg, const double2 *__restrict__ tw, int tw_log) {
    const int n = 1 << lg;
    for (int s = 1; s <= lg; s++) {
        const int half = 1 << (s - 1);
        const int tsh = tw_log - s;
        for (int j = threadIdx.x; j < n / 2; j += blockDim.x) {
            const int pos = j & (half - 1);
            const int i0 = ((j >> (s - 1)) << s) + pos;
            const int i1 = i0 + half;
            const double2 w = tw[pos << tsh];
            const double2 t = cmul(a[i1], w);
            const double2 x0 = a[i0];
            a[i0] = cadd(x0, t);
            a[i1] = csub(x0, t);
        }
        __syncthreads();
    }
}

// In-place radix-2 decimation-in-frequency DFT, natural input, bit-reversed
// output, sign -1 (forward).
__device__ void fft_dif_fwd(double2 *a, int lg, const double2 *__restrict__ tw, int tw_log) {
    const int n = 1 << lg;
    for (int s = lg; s >= 1; s--) {
        const int half = 1 << (s - 1);
        const int tsh = tw_log - s;
        for (int j = threadIdx.x; j < n / 2; j += blockDim.x) {
            const int pos = j & (half - 1);
            const int i0 = ((j >> (s - 1)) << s) + pos;
            const int i1 = i0 + half;
            const double2 w = cconj(tw[pos << tsh]);
            const double2 x0 = a[i0], x1 = a[i1];
            a[i0] = cadd(x0, x1);
            a[i1] = cmul(csub(x0, x1), w);
        }
        __syncthreads();
    }
}

// Raw wrap sum for bin b (without the common phase e^{i pi b s/J}) over the
// residue-class terms j = g, g+G, ... of both classes.
__device__ __forceinline__ double2 gather_bin(const double2 *__restrict__ qr, size_t qstride, int L,
                                              int J, int s, int b, int g, int G) {
    double2 acc = make_double2(0.0, 0.0);
    if (b == 0 && g == 0) acc.x = qr[0].x;  // m = 0: real part only
    for (int j = g;; j += G) {               // m = b + jJ
        long long m = (long long)b + (long long)j * J;
        if (m > L) break;
        if (m == 0) continue;
        double2 v = qr[(size_t)m * qstride];
        if (s & j & 1) v = make_double2(-v.x, -v.y);
        acc = cadd(acc, v);
    }
    for (int j = (g == 0 ? G : g);; j += G) {  // m = jJ - b, j >= 1
        long long m = (long long)j * J - b;
        if (m > L) break;
        double2 v = cconj(qr[(size_t)m * qstride]);
        if (s & j & 1) v = make_double2(-v.x, -v.y);
        acc = cadd(acc, v);
    }
    return acc;
}

__global__ __launch_bounds__(kRingThreads) void k_ring_synth(RingArgs a) {
    extern __shared__ double2 sm[];
    const int item = xcd_item(blockIdx.x);
    if (item >= a.count * a.nmaps) return;
    const int pos = item / a.nmaps, b = item % a.nmaps;
    const int rho = a.rings[pos];
    const int J = a.ring_J[rho], s = a.ring_s[rho], M = a.ring_M[rho];
    const int n = J / 2, lgn = ilog2_dev(n);
    const bool bs = M > 0;
    const int S = bs ? M : n, lgS = ilog2_dev(S);
    double2 *buf = sm;
    double2 *part = sm + S;  // kRingThreads * 2 entries
    const double2 *qr = a.q + (size_t)rho * a.nmaps + b;
    const size_t qstride = (size_t)a.nrings * a.nmaps;
    const int T = blockDim.x, tid = threadIdx.x;

    if (bs)
        for (int i = n + tid; i < M; i += T) buf[i] = make_double2(0.0, 0.0);

    // Z_k for the pair (k, n-k) from the Hermitian bins X_k, X_{n-k}
    auto emit = [&](int k, double2 rk, double2 rnk) {
        double2 Xk = rk, Xnk = rnk;
        if (s) {
            Xk = cmul(Xk, expipi((double)k / J));
            Xnk = cmul(Xnk, expipi((double)(n - k) / J));
        }
        double2 Zk, Znk;
        bool two = (k != 0) && (2 * k != n);
        if (k == 0) {
            double2 e = cadd(Xk, cconj(Xnk)), o = csub(Xk, cconj(Xnk));
            Zk = make_double2(e.x - o.y, e.y + o.x);
        } else if (2 * k == n) {
            Zk = make_double2(2.0 * Xk.x, -2.0 * Xk.y);
        } else {
            double2 e = cadd(Xk, cconj(Xnk));
            double2 o = cmul(csub(Xk, cconj(Xnk)), expipi((double)k / n));
            Zk = make_double2(e.x - o.y, e.y + o.x);
            Znk = make_double2(e.x + o.y, -e.y + o.x);  // conj(e) + i conj(o)
        }
        if (!bs) {
            buf[bitrev(k, lgn)] = Zk;
            if (two) buf[bitrev(n - k, lgn)] = Znk;
        } else {
            long long r = ((long long)k * k) % (2LL * n);
            buf[k] = cmul(Zk, expipi((double)r / n));
            if (two) {
                long long r2 = ((long long)(n - k) * (n - k)) % (2LL * n);
                buf[n - k] = cmul(Znk, expipi((double)r2 / n));
            }
        }
    };

    const int npair = n / 2 + 1;
    if (npair * 2 >= T) {
        for (int k = tid; k < npair; k += T)
            emit(k, gather_bin(qr, qstride, a.L, J, s, k, 0, 1),
                 gather_bin(qr, qstride, a.L, J, s, n - k, 0, 1));
    } else {
        const int G = T / npair;
        const int g = tid / npair, k = tid % npair;
        if (g < G) {
            part[2 * (g * npair + k)] = gather_bin(qr, qstride, a.L, J, s, k, g, G);
            part[2 * (g * npair + k) + 1] = gather_bin(qr, qstride, a.L, J, s, n - k, g, G);
        }
        __syncthreads();
        if (tid < npair) {
            double2 x0 = make_double2(0.0, 0.0), x1 = make_double2(0.0, 0.0);
            for (int gg = 0; gg < G; gg++) {
                x0 = cadd(x0, part[2 * (gg * npair + tid)]);
                x1 = cadd(x1, part[2 * (gg * npair + tid) + 1]);
            }
            emit(tid, x0, x1);
        }
    }
    __syncthreads();

    if (!bs) {
        fft_dit_inv(buf, lgn, a.tw, a.tw_log);
    } else {
        fft_dif_fwd(buf, lgS, a.tw, a.tw_log);
        const double2 *V = a.bs_table + a.ring_bs_off[rho];
        for (int i = tid; i < M; i += T) buf[i] = cmul(buf[i], V[i]);
        __syncthreads();
        fft_dit_inv(buf, lgS, a.tw, a.tw_log);
        for (int p = tid; p < n; p += T) {
            long long r = ((long long)p * p) % (2LL * n);
            buf[p] = cmul(buf[p], expipi((double)r / n));
        }
        __syncthreads();
    }
    // pixel 2p = Re z_p, pixel 2p+1 = Im z_p
    double2 *out = reinterpret_cast<double2 *>(a.map + (size_t)b * a.npix + a.ring_off[rho]);
    for (int p = tid; p < n; p += T) out[p] = buf[p];
}

hipError_t launch_ring_synthesis(const sht_plan_s *p, int nmaps, const double *q, double *map,
                                 hipStream_t stream) {
    RingArgs a;
    a.ring_J = p->d_ring_J;
    a.ring_s = p->d_ring_s;
    a.ring_M = p->d_ring_M;
    a.ring_off = p->d_ring_off;
    a.ring_bs_off = p->d_ring_bs_off;
    a.tw = reinterpret_cast<const double2 *>(p->d_tw);
    a.tw_log = p->tw_log;
    a.bs_table = reinterpret_cast<const double2 *>(p->d_bs_table);
    a.q = reinterpret_cast<const double2 *>(q);
    a.map = map;
    a.L = p->L;
    a.nrings = p->nrings;
    a.nmaps = nmaps;
    a.npix = 12LL * p->nside * p->nside;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_ring_synth, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr_set = true;
    }
    for (const auto &rc : p->classes) {
        a.rings = rc.d_rings;
        a.count = (int)rc.rings.size();
        long long items = (long long)a.count * nmaps;
        long long grid = (items + 63) / 64 * 64;
        size_t lds = (size_t)(rc.lds_entries + 2 * kRingThreads) * sizeof(double2);
        hipLaunchKernelGGL(k_ring_synth, dim3((unsigned)grid), dim3(kRingThreads), lds, stream, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sht
