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
// One workgroup handles one (ring, map).  Bin b collects the m of its two
// residue classes m = b + jJ and m = jJ - b; all of them share the phase
// e^{i pi b s/J} up to the sign (-1)^{js}, so each bin needs one sincospi.
// Rings with J/2 > L (no wrap) load their q values straight into registers,
// all loads in flight at once; so do rings with J > L, whose bins collect
// at most two orders.  Shorter rings sum the orders of each bin straight
// from q as well, several threads per bin when the ring has fewer bins than
// the workgroup has threads, and reduce those partial sums through LDS in a
// fixed order (deterministic, no atomics).  The
// half-length DFT runs in LDS with in-place radix-8 passes (radix-4/2 for the
// remainder): decimation in time on bit-reversed input when n is a power of
// two.  Otherwise n = 2h (J is a multiple of 4) and the DFT is split into its
// even- and odd-index halves, two length-h DFTs run one after the other in
// the same buffer by Bluestein's chirp convolution with a power-of-two
// M >= 2h-1 (forward decimation in frequency, pointwise product with the
// plan's chirp spectrum, backward decimation in time), the first result
// waiting in registers; z_p = A_p + w^p B_p, z_{p+h} = A_p - w^p B_p with
// w = e^{2 pi i/n}.  This halves the LDS of the longest polar rings.  The
// zero padding of each convolution input is implied (the first forward pass
// reads the entries past h as zeros), so it is never stored.  LDS indices
// are padded by one entry per 16 to spread strided accesses over the banks.
// Global loads (q columns, chirps, chirp spectra, pixels) are issued in
// batches before their first use, so that a thread waits for memory once per
// batch rather than once per value.  One workgroup
// owns one (ring, map); the maps of a ring are adjacent in the ring-major q
// layout and their workgroups run back to back on the same XCD (dispatch is
// round-robin over 8 XCDs), so lines read from HBM serve them all from L2.
#include <mutex>
#include <set>
#include <utility>

#include <cstring>

#include "internal.h"

namespace sht {

constexpr int kMaxPairs = 2049;     // Hermitian bin pairs of the largest ring (n = 4096)
constexpr int kMaxHalf = 2048;      // half length h of the largest Bluestein ring (n = 2h <= 4096)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// Complex product with a fixed rounding pattern (explicit fused multiply-adds)
// for the chirp products, whose loops take different shapes in different
// kernels (batched loads or one at a time): whichever way the compiler would
// contract the plain expression there, the ring kernels of one plan (one map
// per workgroup, several, or the batch queue) agree bit for bit.
__device__ __forceinline__ double2 cmul_fixed(double2 a, double2 b) {
    return make_double2(__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 expipi(double x) {  // e^{i pi x}
    double s, c;
    sincospi(x, &s, &c);
    return make_double2(c, s);
}
// x * i conj(y): with y = e^{i pi k/J} and n = J/2, e^{i pi (n - k)/J} = i conj(y)
__device__ __forceinline__ double2 i_conj(double2 y) { return make_double2(y.y, y.x); }
__device__ __forceinline__ int ilog2_dev(int n) { return 31 - __clz(n); }
__device__ __forceinline__ int bitrev(int k, int lg) { return lg == 0 ? 0 : (int)(__brev((unsigned)k) >> (32 - lg)); }
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

// Workgroup -> work item, grouping 8 consecutive items on one XCD.
__device__ __forceinline__ int xcd_item(int wg) { return (wg & ~63) + ((wg & 7) << 3) + ((wg >> 3) & 7); }

// x * e^{2 pi i j / 8} for j = 0..7 (exact constants)
__device__ __forceinline__ double2 rot8(double2 x, int j) {
    const double r = 0.70710678118654752440;
    switch (j & 7) {
        case 0: return x;
        case 1: return make_double2(r * (x.x - x.y), r * (x.x + x.y));
        case 2: return make_double2(-x.y, x.x);
        case 3: return make_double2(-r * (x.x + x.y), r * (x.x - x.y));
        case 4: return make_double2(-x.x, -x.y);
        case 5: return make_double2(r * (x.y - x.x), -r * (x.x + x.y));
        case 6: return make_double2(x.y, -x.x);
        default: return make_double2(r * (x.x + x.y), r * (x.y - x.x));
    }
}

// One in-place pass of 2^r radix-2 stages s .. s+r-1 (h = 2^(s-1)).
// Decimation in time, sign +1 (backward): within each group of R = 2^r
// elements base + k h, sub-stage u combines k and k + 2^u with the twiddle
// e^{+2 pi i (pos + j h) / (2^(u+1) h)}, j = k mod 2^u.
template <int r>
__device__ __forceinline__ void dit_pass(double2 *a, int lg, int s, const double2 *__restrict__ tw,
                                         int tw_log, int tid, int nt) {
    constexpr int R = 1 << r;
    const int n = 1 << lg, h = 1 << (s - 1);
#pragma unroll 1
    for (int gi = tid; gi < n / R; gi += nt) {
        const int pos = gi & (h - 1);
        const int base = (gi >> (s - 1)) * (R * h) + pos;
        double2 x[R];
#pragma unroll
        for (int k = 0; k < R; k++) x[k] = a[pidx(base + k * h)];
        double2 wp[r];                             // wp[u] = e^{2 pi i pos / (2^(u+1) h)}
        wp[r - 1] = tw[pos << (tw_log - (s - 1) - r)];
#pragma unroll
        for (int u = r - 2; u >= 0; u--) wp[u] = cmul(wp[u + 1], wp[u + 1]);
#pragma unroll
        for (int u = 0; u < r; u++) {
            const int span = 1 << u;
#pragma unroll
            for (int k = 0; k < R; k++) {
                if (k & span) continue;
                const int j = k & (span - 1);
                const double2 w = rot8(wp[u], j * (4 >> u));  // e^{2 pi i j / 2^(u+1)}
                const double2 t = cmul(x[k + span], w);
                x[k + span] = csub(x[k], t);
                x[k] = cadd(x[k], t);
            }
        }
#pragma unroll
        for (int k = 0; k < R; k++) a[pidx(base + k * h)] = x[k];
    }
    __syncthreads();
}

// Decimation in frequency, sign -1 (forward): the same groups with the
// sub-stages in reverse order and conjugate twiddles applied after the
// difference.
template <int r>
__device__ __forceinline__ void dif_pass(double2 *a, int lg, int s, const double2 *__restrict__ tw,
                                         int tw_log, int tid, int nt, int nz) {
    constexpr int R = 1 << r;
    const int n = 1 << lg, h = 1 << (s - 1);
#pragma unroll 1
    for (int gi = tid; gi < n / R; gi += nt) {
        const int pos = gi & (h - 1);
        const int base = (gi >> (s - 1)) * (R * h) + pos;
        double2 x[R];
#pragma unroll
        for (int k = 0; k < R; k++) x[k] = base + k * h < nz ? a[pidx(base + k * h)] : make_double2(0.0, 0.0);
        double2 wp[r];
        wp[r - 1] = tw[pos << (tw_log - (s - 1) - r)];
#pragma unroll
        for (int u = r - 2; u >= 0; u--) wp[u] = cmul(wp[u + 1], wp[u + 1]);
#pragma unroll
        for (int u = r - 1; u >= 0; u--) {
            const int span = 1 << u;
#pragma unroll
            for (int k = 0; k < R; k++) {
                if (k & span) continue;
                const int j = k & (span - 1);
                const double2 w = cconj(rot8(wp[u], j * (4 >> u)));
                const double2 x0 = x[k], x1 = x[k + span];
                x[k] = cadd(x0, x1);
                x[k + span] = cmul(csub(x0, x1), w);
            }
        }
#pragma unroll
        for (int k = 0; k < R; k++) a[pidx(base + k * h)] = x[k];
    }
    __syncthreads();
}

// Backward DFT of size 2^lg, bit-reversed input, natural output, by the nt
// threads tid = 0..nt-1 of the caller's thread group.
__device__ void fft_dit_inv(double2 *a, int lg, const double2 *__restrict__ tw, int tw_log, int tid, int nt) {
    int s = 1;
    while (lg - s + 1 >= 3) {
        dit_pass<3>(a, lg, s, tw, tw_log, tid, nt);
        s += 3;
    }
    if (lg - s + 1 == 2) dit_pass<2>(a, lg, s, tw, tw_log, tid, nt);
    else if (lg - s + 1 == 1) dit_pass<1>(a, lg, s, tw, tw_log, tid, nt);
}

// Forward DFT of size 2^lg, natural input, bit-reversed output; the inputs
// past the first nz are zero (the first pass reads them as such, so they
// need not be stored).
__device__ void fft_dif_fwd(double2 *a, int lg, const double2 *__restrict__ tw, int tw_log, int tid, int nt,
                            int nz) {
    const int n = 1 << lg, rem = lg % 3;
    int s = lg - 2;
    while (s >= 1 + rem) {
        dif_pass<3>(a, lg, s, tw, tw_log, tid, nt, s == lg - 2 ? nz : n);
        s -= 3;
    }
    if (rem == 2) dif_pass<2>(a, lg, 1, tw, tw_log, tid, nt, lg == 2 ? nz : n);
    else if (rem == 1) dif_pass<1>(a, lg, 1, tw, tw_log, tid, nt, lg == 1 ? nz : n);
}

// buf[pidx(i)] *= X[i] for the entries i = tid + j nt < cnt (j < PT) of one
// thread, up to NB loads of X in flight before the first product (loads
// past cnt read X[cnt - 1] and are dropped).
template <int PT, int NB>
__device__ __forceinline__ void lds_cmul(double2 *buf, const double2 *__restrict__ X, int cnt, int tid, int nt) {
    constexpr int B = PT < NB ? PT : NB;
    if (B == 1) {  // one load at a time
        for (int i = tid; i < cnt; i += nt) buf[pidx(i)] = cmul_fixed(buf[pidx(i)], X[i]);
        return;
    }
#pragma unroll
    for (int j0 = 0; j0 < PT; j0 += B) {
        double2 x[B];
#pragma unroll
        for (int j = 0; j < B; j++) x[j] = X[min(tid + (j0 + j) * nt, cnt - 1)];
#pragma unroll
        for (int j = 0; j < B; j++) {
            const int i = tid + (j0 + j) * nt;
            if (i < cnt) buf[pidx(i)] = cmul_fixed(buf[pidx(i)], x[j]);
        }
    }
}

// Unnormalised backward DFT of size n in LDS: z_p = sum_k Z_k e^{+2 pi i k p/n}.
// On entry the buffer holds Z_k at pidx(bitrev(k)) (n a power of two, M = 0)
// or the chirp-weighted u_k = Z_k W_k, W_k = e^{i pi k^2/n}, at pidx(k), k < n
// (Bluestein: the zero padding up to M is implied, entries n..M-1 are not
// read); on exit z_p is at pidx(p), p < n.  PT bounds M / nt (and so
// 2n / nt); NB loads of V or W per thread are in flight at once.
template <int PT, int NB>
__device__ __forceinline__ void backward_dft(double2 *buf, int n, int M, const double2 *__restrict__ V,
                                             const double2 *__restrict__ W, const double2 *__restrict__ tw,
                                             int tw_log, int tid, int nt) {
    if (M == 0) {
        fft_dit_inv(buf, ilog2_dev(n), tw, tw_log, tid, nt);
        return;
    }
    const int lgM = ilog2_dev(M);
    fft_dif_fwd(buf, lgM, tw, tw_log, tid, nt, n);
    lds_cmul<PT, NB>(buf, V, M, tid, nt);
    __syncthreads();
    fft_dit_inv(buf, lgM, tw, tw_log, tid, nt);
    lds_cmul<(PT > 1 ? PT / 2 : 1), NB>(buf, W, n, tid, nt);
    __syncthreads();
}

// Raw wrap sums (before the common phase) of the NBIN bins bin[p] of one
// thread (bins with on[p] false give 0) over every order, restricted to the
// terms j = g (mod G): class 1 m = b + jJ (j >= 0), then class 2 m = jJ - b
// (j >= 1), each in increasing j, read straight from the ring's q column
// (stride qs).  Loads go in rounds of U terms of every bin: all of a round's
// loads are issued before the first is added (loads past a bin's last term
// take order 0 and are dropped), so a thread waits for memory once per
// round rather than once per term.
template <int NBIN, int U>
__device__ __forceinline__ void bins_direct(const double2 *__restrict__ qr, size_t qs, int L, int J, int s,
                                            const int (&bin)[NBIN], const bool (&on)[NBIN], int g, int G,
                                            double2 (&acc)[NBIN]) {
    const int g2 = g == 0 ? G : g;  // first j of class 2
    int c1[NBIN], c2[NBIN];         // terms of each class (m <= L: j <= (L -+ b) / J)
    int r1 = 0, r2 = 0;
#pragma unroll
    for (int p = 0; p < NBIN; p++) {
        acc[p] = make_double2(0.0, 0.0);
        const int j1 = (L - bin[p]) / J, j2 = (L + bin[p]) / J;
        c1[p] = on[p] && j1 >= g ? (j1 - g) / G + 1 : 0;
        c2[p] = on[p] && j2 >= g2 ? (j2 - g2) / G + 1 : 0;
        r1 = max(r1, c1[p]);
        r2 = max(r2, c2[p]);
    }
    for (int i0 = 0; i0 < r1; i0 += U) {
        double2 v[NBIN][U];
#pragma unroll
        for (int p = 0; p < NBIN; p++)
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int i = min(i0 + u, c1[p] - 1);
                v[p][u] = qr[(size_t)(i < 0 ? 0 : bin[p] + (g + i * G) * J) * qs];
            }
#pragma unroll
        for (int p = 0; p < NBIN; p++)
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int j = g + (i0 + u) * G;
                if (i0 + u < c1[p]) {
                    double2 x = v[p][u];
                    if (bin[p] + j * J == 0) x.y = 0.0;  // real part of q_0 only
                    if (s & j & 1) x = make_double2(-x.x, -x.y);
                    acc[p] = cadd(acc[p], x);
                }
            }
    }
    for (int i0 = 0; i0 < r2; i0 += U) {
        double2 v[NBIN][U];
#pragma unroll
        for (int p = 0; p < NBIN; p++)
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int i = min(i0 + u, c2[p] - 1);
                v[p][u] = qr[(size_t)(i < 0 ? 0 : (g2 + i * G) * J - bin[p]) * qs];
            }
#pragma unroll
        for (int p = 0; p < NBIN; p++)
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int j = g2 + (i0 + u) * G;
                if (i0 + u < c2[p]) {
                    double2 x = cconj(v[p][u]);
                    if (s & j & 1) x = make_double2(-x.x, -x.y);
                    acc[p] = cadd(acc[p], x);
                }
            }
    }
}

// Synthesis of one ring of one map (item = ring position in the class's
// list times nmaps plus the map) by the nt threads tid = 0..nt-1 of a group
// owning the LDS block buf.  A workgroup of T threads is one group, or T/nt
// groups for maps of one ring (identical control flow, so the workgroup's
// barriers match); a ring whose transform size is at most 4096 nt / T keeps
// the per-thread counts within those sized for T.
template <int T, int nt, int kNB>
__device__ __forceinline__ void ring_synth_item(const RingArgs &a, const int item, const int tid, double2 *buf) {
    constexpr int kPairsPerThread = (kMaxPairs + T - 1) / T;
    constexpr int kMPerThread = (2 * kMaxHalf + T - 1) / T;  // Bluestein size M <= 2 kMaxHalf
    const int pos = item / a.nmaps, b = item % a.nmaps;
    const int rho = a.rings[pos];
    const int J = a.ring_J[rho], s = a.ring_s[rho], M = a.ring_M[rho];
    const int n = J / 2, lgn = ilog2_dev(n);
    const bool bs = M > 0;
    const double2 *__restrict__ W = a.chirp + (bs ? a.ring_chirp_off[rho] : 0);
    const int L = a.L;
    const int npair = n / 2 + 1;
    // ring-major q: the maps of one ring interleave in one contiguous block,
    // and their workgroups run back to back on one XCD (shared L2 lines)
    const size_t qstride = (size_t)a.nmaps;
    const double2 *qr = a.q + (size_t)rho * (L + 1) * a.nmaps + b;

    // raw bin sums for the pairs (k, n-k) owned by this thread
    double2 xa[kPairsPerThread], xb[kPairsPerThread];
#pragma unroll
    for (int j = 0; j < kPairsPerThread; j++) xa[j] = xb[j] = make_double2(0.0, 0.0);

    const bool wrap = n <= L;
    int G = 1;
    if (!wrap) {
        // every bin b <= L holds exactly q_b; issue all loads first
#pragma unroll
        for (int j = 0; j < kPairsPerThread; j++) {
            const int k = tid + j * nt;
            if (k < npair) {
                if (k <= L) xa[j] = qr[(size_t)k * qstride];
                if (k == 0) xa[j].y = 0.0;
                if (k != 0 && n - k <= L) xb[j] = qr[(size_t)(n - k) * qstride];
            }
        }
    } else if (2 * n > L) {
        // J > L: bin b <= n collects m = b and, when J - b <= L, m = J - b
        // (conjugated, sign (-1)^s); bin n (pair k = 0) collects m = n
        // (j = 0) and m = J - n = n (j = 1, conjugated).  Direct loads, no
        // staging: the four loads of every pair of a chunk of kCH pairs are
        // issued (at valid orders) before any is used, and the optional
        // terms enter by selection
        const double sg = (s & 1) ? -1.0 : 1.0;
        const int J2 = 2 * n;
        constexpr int kCH = kPairsPerThread < 3 ? kPairsPerThread : 3;
#pragma unroll
        for (int j0 = 0; j0 < kPairsPerThread; j0 += kCH) {
            double2 v[kCH][4];
#pragma unroll
            for (int c = 0; c < kCH; c++) {
                const int k = tid + (j0 + c) * nt;
                const int kc = j0 + c < kPairsPerThread && k < npair ? k : 0;
                const int b = kc == 0 ? n : n - kc;  // second bin, 0 < b <= n
                v[c][0] = qr[(size_t)kc * qstride];  // kc <= n <= L
                v[c][1] = qr[(size_t)(J2 - kc <= L ? J2 - kc : 0) * qstride];
                v[c][2] = qr[(size_t)b * qstride];
                v[c][3] = qr[(size_t)(kc == 0 ? n : (J2 - b <= L ? J2 - b : 0)) * qstride];
            }
#pragma unroll
            for (int c = 0; c < kCH; c++) {
                const int j = j0 + c, k = tid + j * nt;
                if (j < kPairsPerThread && k < npair) {
                    const int b = k == 0 ? n : n - k;
                    double2 x = v[c][0];
                    if (k == 0) x.y = 0.0;
                    const double2 xw = make_double2(x.x + sg * v[c][1].x, x.y - sg * v[c][1].y);
                    xa[j] = J2 - k <= L ? xw : x;
                    const double2 u = v[c][2];
                    const double2 uw = make_double2(u.x + sg * v[c][3].x, u.y - sg * v[c][3].y);
                    xb[j] = k == 0 || J2 - b <= L ? uw : u;
                }
            }
            asm volatile("" ::: "memory");  // keep the next chunk's loads after this one's uses
        }
    } else {
        // J <= L: every bin collects several orders; each thread sums the
        // orders of its bins (terms j = g mod G) straight from q, in a fixed
        // order: pair k owns bins k and n - k (bin n for k = 0, none for
        // 2k = n)
        G = npair >= nt ? 1 : nt / npair;
        if (npair <= nt) {
            // one pair per thread (G groups of npair threads), four terms
            // of each bin per round of loads
            const int g = tid / npair, k = tid % npair;
            const int bn[2] = {k, k == 0 ? n : n - k};
            const bool on[2] = {g < G, g < G && 2 * k != n};
            double2 acc[2];
            bins_direct<2, 4>(qr, qstride, L, J, s, bn, on, g, G, acc);
            xa[0] = acc[0];
            xb[0] = acc[1];
        } else {
            // several pairs per thread (G = 1): rounds of one term of each
            // of up to 2 kCP bins
            constexpr int kCP = kPairsPerThread < 3 ? kPairsPerThread : 3;
#pragma unroll
            for (int j0 = 0; j0 < kPairsPerThread; j0 += kCP) {
                int bn[2 * kCP];
                bool on[2 * kCP];
#pragma unroll
                for (int c = 0; c < kCP; c++) {
                    const int k = tid + (j0 + c) * nt;
                    bn[2 * c] = k;
                    bn[2 * c + 1] = k == 0 ? n : n - k;
                    on[2 * c] = j0 + c < kPairsPerThread && k < npair;
                    on[2 * c + 1] = on[2 * c] && 2 * k != n;
                }
                double2 acc[2 * kCP];
                bins_direct<2 * kCP, 1>(qr, qstride, L, J, s, bn, on, 0, 1, acc);
#pragma unroll
                for (int c = 0; c < kCP; c++)
                    if (j0 + c < kPairsPerThread) {
                        xa[j0 + c] = acc[2 * c];
                        xb[j0 + c] = acc[2 * c + 1];
                    }
            }
        }
        if (G > 1) {
            // reduce the group partials in a fixed order, through the start
            // of the group's LDS block (at least 2 nt entries), before the
            // DFT uses it
            double2 *red = buf;
            if (tid < G * npair) {
                red[2 * tid] = xa[0];
                red[2 * tid + 1] = xb[0];
            }
            __syncthreads();
            if (tid < npair) {
                double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
                for (int g = 0; g < G; g++) {
                    s0 = cadd(s0, red[2 * (g * npair + tid)]);
                    s1 = cadd(s1, red[2 * (g * npair + tid) + 1]);
                }
                xa[0] = s0;
                xb[0] = s1;
            }
            __syncthreads();
        }
    }

    // phase shift, Hermitian pre-twiddle, store into the DFT input: natural
    // bit-reversed order for power-of-two n; for split Bluestein rings even k
    // at k/2 and odd k at h + (k-1)/2 (n = 2h), weighted by the chirp
    const int h = n / 2;
    // e^{i pi k/J} and e^{i pi k/n} for k = tid + j nt by products with the
    // step e^{i pi nt/J} (resp. n): two sincospi per thread instead of three
    // per pair (the rounding grows by about an ulp per step)
    double2 pJ = make_double2(1.0, 0.0), sJ = pJ;
    if (s) {
        pJ = expipi((double)tid / J);
        sJ = expipi((double)nt / J);
    }
    double2 pn = expipi((double)tid / n);
    const double2 sn = expipi((double)nt / n);
    // Bluestein chirp weights W[kp], W[kq] of a chunk of kCW pairs loaded
    // (at clamped, valid indices) before the chunk's first use
    constexpr int kCW = kPairsPerThread < 3 ? kPairsPerThread : 3;
#pragma unroll
    for (int j0 = 0; j0 < kPairsPerThread; j0 += kCW) {
    double2 wv[kCW][2];
    if (bs) {
#pragma unroll
        for (int c = 0; c < kCW; c++) {
            const int k = tid + (j0 + c) * nt, odd = k & 1;
            wv[c][0] = W[max(0, min((k - odd) / 2, h - 1))];
            wv[c][1] = W[max(0, min((n - k - odd) / 2, h - 1))];
        }
    }
#pragma unroll
    for (int c = 0; c < kCW; c++) {
        const int j = j0 + c;
        if (j >= kPairsPerThread) break;
        const int k = tid + j * nt;
        if (k < npair && !(G > 1 && j > 0)) {
        double2 Xk = xa[j], Xnk = xb[j];
        if (s) {
            Xk = cmul(Xk, pJ);
            Xnk = cmul(Xnk, i_conj(pJ));  // e^{i pi (n - k)/J}, n = J/2
        }
        double2 Zk, Znk = make_double2(0.0, 0.0);
        const bool two = (k != 0) && (2 * k != n);
        if (k == 0) {
            double2 e = cadd(Xk, cconj(Xnk)), o = csub(Xk, cconj(Xnk));
            Zk = make_double2(e.x - o.y, e.y + o.x);
        } else if (2 * k == n) {
            Zk = make_double2(2.0 * Xk.x, -2.0 * Xk.y);
        } else {
            double2 e = cadd(Xk, cconj(Xnk));
            double2 o = cmul(csub(Xk, cconj(Xnk)), pn);
            Zk = make_double2(e.x - o.y, e.y + o.x);
            Znk = make_double2(e.x + o.y, -e.y + o.x);  // conj(e) + i conj(o)
        }
        if (!bs) {
            buf[pidx(bitrev(k, lgn))] = Zk;
            if (two) buf[pidx(bitrev(n - k, lgn))] = Znk;
        } else {
            const int odd = k & 1, kp = (k - odd) / 2;
            buf[pidx(kp + odd * h)] = cmul(Zk, wv[c][0]);
            if (two) {
                const int kq = (n - k - odd) / 2;
                buf[pidx(kq + odd * h)] = cmul(Znk, wv[c][1]);
            }
        }
        }
        pJ = cmul(pJ, sJ);
        pn = cmul(pn, sn);
    }
    }
    __syncthreads();
    // pixel 2p = Re z_p, pixel 2p+1 = Im z_p
    double2 *out = reinterpret_cast<double2 *>(a.map + (size_t)b * a.npix + a.ring_off[rho]);
    if (!bs) {
        backward_dft<kMPerThread, kNB>(buf, n, 0, nullptr, nullptr, a.tw, a.tw_log, tid, nt);
        for (int p = tid; p < n; p += nt) out[p] = buf[pidx(p)];
        return;
    }

    // split Bluestein: the odd half waits in registers while the even half
    // (A) is transformed, then A waits while the odd half (B) is
    constexpr int kHalfPerThread = (kMaxHalf + T - 1) / T;
    const double2 *__restrict__ V = a.bs_table + a.ring_bs_off[rho];
    double2 R[kHalfPerThread];
#pragma unroll
    for (int jj = 0; jj < kHalfPerThread; jj++) {
        const int p = tid + jj * nt;
        if (p < h) R[jj] = buf[pidx(h + p)];
    }
    __syncthreads();
    backward_dft<kMPerThread, kNB>(buf, h, M, V, W, a.tw, a.tw_log, tid, nt);
#pragma unroll
    for (int jj = 0; jj < kHalfPerThread; jj++) {
        const int p = tid + jj * nt;
        if (p < h) {
            const double2 odd_in = R[jj];
            R[jj] = buf[pidx(p)];  // A_p
            buf[pidx(p)] = odd_in;
        }
    }
    __syncthreads();
    backward_dft<kMPerThread, kNB>(buf, h, M, V, W, a.tw, a.tw_log, tid, nt);
    double2 wp = expipi(2.0 * tid / n);  // e^{2 pi i p/n}, stepped as above
    const double2 ws = expipi(2.0 * nt / n);
#pragma unroll
    for (int jj = 0; jj < kHalfPerThread; jj++) {
        const int p = tid + jj * nt;
        if (p < h) {
            const double2 t = cmul(buf[pidx(p)], wp);
            out[p] = cadd(R[jj], t);
            out[p + h] = csub(R[jj], t);
        }
        wp = cmul(wp, ws);
    }
}

// Workgroup w runs the items w G .. w G + G - 1 (G = a.mpw maps of one
// ring, G | nmaps), one group of T/G threads and one LDS block each.
template <int T, int G>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(T == 512 ? 4 : 1))) void k_ring_synth(RingArgs a) {
    extern __shared__ double2 sm[];
    constexpr int nt = T / G;
    const int sub = G == 1 ? 0 : (int)threadIdx.x / nt;
    const int item0 = xcd_item(blockIdx.x) * G;
    if (item0 >= a.count * a.nmaps) return;
    // (one group: the plain thread index and LDS base keep 26 fewer VGPRs)
    if (G == 1) ring_synth_item<T, nt, (T >= 512 ? 8 : 1)>(a, item0, threadIdx.x, sm);
    else ring_synth_item<T, nt, 1>(a, item0 + sub, threadIdx.x - sub * nt, sm + (size_t)sub * (a.fft_entries + a.stage));
}

// Ring queue of a batch of requests: one launch per ring size class for all
// requests, item j = {argument block (request, class), item of that class};
// items are ordered request by request, ring by ring, map by map, so that
// the maps of one ring stay on one XCD as in k_ring_synth.
template <int T>
__global__ __launch_bounds__(T) void k_ring_synth_queue(const RingArgs *__restrict__ args, const int2 *__restrict__ items,
                                                        int nitems) {
    const int j = xcd_item(blockIdx.x);
    if (j >= nitems) return;
    const int2 it = items[j];
    extern __shared__ double2 sm[];
    const RingArgs a = args[__builtin_amdgcn_readfirstlane(it.x)];
    ring_synth_item<T, T, 1>(a, __builtin_amdgcn_readfirstlane(it.y), threadIdx.x, sm);
}

// Raises a kernel's dynamic LDS limit to `bytes`, once per (kernel, device):
// the attribute belongs to the device current at the call.
hipError_t allow_dynamic_lds(const void *fn, int bytes) {
    static std::mutex mu;
    static std::set<std::pair<const void *, int>> done;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    if (done.count({fn, dev})) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) done.insert({fn, dev});
    return e;
}

// FFT buffer entries, extra entries and dynamic LDS bytes of the workgroups
// of one ring class (FFT buffer of lds_entries complex values) at T threads:
// wrapped rings reduce up to 2 T partial bin sums through the start of the
// block, so the block holds at least 2 T entries.
size_t ring_class_shape(int lds_entries, bool wrap, int T, int *fft_entries, int *stage) {
    *fft_entries = lds_entries + lds_entries / 16;
    *stage = wrap ? std::max(0, 2 * T - *fft_entries) : 0;
    return (size_t)(*fft_entries + *stage) * sizeof(double2);
}

// Maps of one ring per workgroup for a class of transform size S: as many
// as fill the workgroup's threads with the groups a 4096-entry transform
// would use (at most 4), dividing nmaps.
int ring_maps_per_wg(int lds_entries, int nmaps) {
    int g = 1;
    while (g < 4 && (g * 2) * lds_entries <= 4096 && nmaps % (g * 2) == 0) g *= 2;
    return g;
}

template <int T>
static hipError_t launch_classes(const sht_plan_s *p, RingArgs a, int nmaps, hipStream_t stream) {
    const void *fn[3] = {(const void *)k_ring_synth<T, 1>, (const void *)k_ring_synth<T, 2>,
                         (const void *)k_ring_synth<T, 4>};
    for (const void *f : fn) {
        hipError_t ea = allow_dynamic_lds(f, 160 * 1024);
        if (ea != hipSuccess) return ea;
    }
    for (const auto &rc : p->classes) {
        a.rings = rc.d_rings;
        a.count = (int)rc.rings.size();
        a.mpw = ring_maps_per_wg(rc.lds_entries, nmaps);
        const size_t lds = a.mpw * ring_class_shape(rc.lds_entries, rc.wrap, T / a.mpw, &a.fft_entries, &a.stage);
        long long grid = ((long long)a.count * nmaps / a.mpw + 63) / 64 * 64;
        switch (a.mpw) {
            case 1: hipLaunchKernelGGL((k_ring_synth<T, 1>), dim3((unsigned)grid), dim3(T), lds, stream, a); break;
            case 2: hipLaunchKernelGGL((k_ring_synth<T, 2>), dim3((unsigned)grid), dim3(T), lds, stream, a); break;
            default: hipLaunchKernelGGL((k_ring_synth<T, 4>), dim3((unsigned)grid), dim3(T), lds, stream, a); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int T>
static hipError_t launch_ring_queue_t(const RingArgs *args, const int2 *items, long long nitems, size_t lds,
                                      hipStream_t st) {
    hipError_t e = allow_dynamic_lds((const void *)k_ring_synth_queue<T>, 160 * 1024);
    if (e != hipSuccess) return e;
    const long long grid = (nitems + 63) / 64 * 64;
    if (grid > 0) hipLaunchKernelGGL(k_ring_synth_queue<T>, dim3((unsigned)grid), dim3(T), lds, st, args, items, (int)nitems);
    return hipGetLastError();
}

// Raises the ring queue kernel's LDS limit on the current device (done at
// batch creation, so that runs make no runtime calls besides launches).
hipError_t ring_queue_prepare(int T) {
    switch (T) {
        case 256: return allow_dynamic_lds((const void *)k_ring_synth_queue<256>, 160 * 1024);
        case 512: return allow_dynamic_lds((const void *)k_ring_synth_queue<512>, 160 * 1024);
        default: return allow_dynamic_lds((const void *)k_ring_synth_queue<1024>, 160 * 1024);
    }
}

hipError_t launch_ring_queue(int T, const RingArgs *args, const int2 *items, long long nitems, size_t lds,
                             hipStream_t st) {
    if (nitems < 0 || nitems > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (T) {
        case 256: return launch_ring_queue_t<256>(args, items, nitems, lds, st);
        case 512: return launch_ring_queue_t<512>(args, items, nitems, lds, st);
        default: return launch_ring_queue_t<1024>(args, items, nitems, lds, st);
    }
}

// Plan-wide fields of the ring argument block (synthesis direction); the
// caller sets the class fields (rings, count, fft_entries, stage).
RingArgs ring_args(const sht_plan_s *p, int nmaps, const double *q, double *map) {
    RingArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ring_J = p->d_ring_J;
    a.ring_s = p->d_ring_s;
    a.ring_M = p->d_ring_M;
    a.ring_off = p->d_ring_off;
    a.ring_bs_off = p->d_ring_bs_off;
    a.tw = reinterpret_cast<const double2 *>(p->d_tw);
    a.tw_log = p->tw_log;
    a.bs_table = reinterpret_cast<const double2 *>(p->d_bs_table);
    a.chirp = reinterpret_cast<const double2 *>(p->d_chirp);
    a.ring_chirp_off = p->d_ring_chirp_off;
    a.q = reinterpret_cast<const double2 *>(q);
    a.map = map;
    a.L = p->L;
    a.nrings = p->nrings;
    a.nmaps = nmaps;
    a.npix = 12LL * p->nside * p->nside;
    a.mpw = 1;
    return a;
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
    a.chirp = reinterpret_cast<const double2 *>(p->d_chirp);
    a.ring_chirp_off = p->d_ring_chirp_off;
    a.q = reinterpret_cast<const double2 *>(q);
    a.map = map;
    a.map_in = nullptr;
    a.ybar = nullptr;
    a.wpos = 0.0;
    a.L = p->L;
    a.nrings = p->nrings;
    a.nmaps = nmaps;
    a.npix = 12LL * p->nside * p->nside;
    switch (p->ring_threads) {
        case 256: return launch_classes<256>(p, a, nmaps, stream);
        case 512: return launch_classes<512>(p, a, nmaps, stream);
        default: return launch_classes<1024>(p, a, nmaps, stream);
    }
    return hipSuccess;
}

// Ring stage of the adjoint (the transpose of the above).  For ring k:
//   ybar_m = w_m sum_j y_j e^{-i m phi_j} = w_m e^{-i pi m s/J} F_{m mod J},
//   F_b = sum_j y_j e^{-2 pi i b j/J}  (F_{J-b} = conj F_b),
// with w_0 = 1 and w_m = wpos for m >= 1.  F_0..F_{J/2} come from one complex
// DFT of half length on z_p = y_{2p} + i y_{2p+1} (forward DFT taken as the
// conjugate of the backward one, so the synthesis FFT code is reused), and
// every m of bin b's two residue classes is written from G_b =
// e^{-i pi b s/J} F_b:  ybar_{b+jJ} = w (-1)^{js} G_b,
// ybar_{jJ-b} = w (-1)^{js} conj(G_b).
// Workgroups of a.mpw maps of one ring, one group of T/a.mpw threads and one
// LDS block each, as in k_ring_synth.
template <int T, int G>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(T == 512 ? 4 : 1))) void k_ring_analysis(RingArgs a) {
    extern __shared__ double2 sm[];
    constexpr int nt = T / G;
    const int sub = G == 1 ? 0 : (int)threadIdx.x / nt;
    const int item0 = xcd_item(blockIdx.x) * G;
    if (item0 >= a.count * a.nmaps) return;
    const int item = item0 + sub;
    const int pos = item / a.nmaps, b = item % a.nmaps;
    const int rho = a.rings[pos];
    const int J = a.ring_J[rho], s = a.ring_s[rho], M = a.ring_M[rho];
    const int n = J / 2, lgn = ilog2_dev(n);
    const bool bs = M > 0;
    const double2 *__restrict__ W = a.chirp + (bs ? a.ring_chirp_off[rho] : 0);
    double2 *buf = G == 1 ? sm : sm + (size_t)sub * a.fft_entries;
    const int tid = G == 1 ? (int)threadIdx.x : (int)threadIdx.x - sub * nt;
    const int L = a.L;
    const size_t qstride = (size_t)a.nmaps;
    double2 *yr = a.ybar + (size_t)rho * (L + 1) * a.nmaps + b;

    const double2 *pix = reinterpret_cast<const double2 *>(a.map_in + (size_t)b * a.npix + a.ring_off[rho]);
    constexpr int kMPerThread = (2 * kMaxHalf + T - 1) / T;  // n / nt, or M / nt for Bluestein rings
    constexpr int kLdMax = G == 1 && T >= 512 ? 8 : 1;  // input loads in flight per thread (registers permitting)
    constexpr int kLd = kMPerThread < kLdMax ? kMPerThread : kLdMax;
    constexpr int kNB = G == 1 && T >= 512 ? 8 : 1;  // chirp loads in flight (registers permitting)
    if (!bs) {
        if (kLd == 1) {
            for (int p = tid; p < n; p += nt) buf[pidx(bitrev(p, lgn))] = cconj(pix[p]);
        } else {
#pragma unroll
            for (int j0 = 0; j0 < kMPerThread; j0 += kLd) {
                double2 x[kLd];
#pragma unroll
                for (int j = 0; j < kLd; j++) x[j] = pix[min(tid + (j0 + j) * nt, n - 1)];
#pragma unroll
                for (int j = 0; j < kLd; j++) {
                    const int p = tid + (j0 + j) * nt;
                    if (p < n) buf[pidx(bitrev(p, lgn))] = cconj(x[j]);
                }
            }
        }
        __syncthreads();
        backward_dft<kMPerThread, kNB>(buf, n, 0, nullptr, nullptr, a.tw, a.tw_log, tid, nt);
    } else {
        // split Bluestein: even inputs (hh = 0), then odd inputs (hh = 1)
        constexpr int kHalfPerThread = (kMaxHalf + T - 1) / T;
        constexpr int kLdH = kHalfPerThread < kLdMax ? kHalfPerThread : kLdMax;
        const int h = n / 2;
        const double2 *__restrict__ V = a.bs_table + a.ring_bs_off[rho];
        double2 A[kHalfPerThread];
        for (int hh = 0; hh < 2; hh++) {
            if (kLdH == 1) {
                for (int p = tid; p < h; p += nt) buf[pidx(p)] = cmul(cconj(pix[2 * p + hh]), W[p]);
            } else {
#pragma unroll
                for (int j0 = 0; j0 < kHalfPerThread; j0 += kLdH) {
                    double2 x[kLdH], w[kLdH];
#pragma unroll
                    for (int j = 0; j < kLdH; j++) {
                        const int pc = min(tid + (j0 + j) * nt, h - 1);
                        x[j] = pix[2 * pc + hh];
                        w[j] = W[pc];
                    }
#pragma unroll
                    for (int j = 0; j < kLdH; j++) {
                        const int p = tid + (j0 + j) * nt;
                        if (p < h) buf[pidx(p)] = cmul(cconj(x[j]), w[j]);
                    }
                }
            }
            __syncthreads();
            backward_dft<kMPerThread, kNB>(buf, h, M, V, W, a.tw, a.tw_log, tid, nt);
            if (hh == 0) {
#pragma unroll
                for (int jj = 0; jj < kHalfPerThread; jj++) {
                    const int p = tid + jj * nt;
                    if (p < h) A[jj] = buf[pidx(p)];
                }
                __syncthreads();
            }
        }
        // Z_p = A_p + w^p B_p and Z_{p+h} = A_p - w^p B_p in place (each
        // thread reads B_p before writing p and p + h, which no other thread
        // reads)
        double2 wp = expipi(2.0 * tid / n);  // e^{2 pi i p/n}, stepped by products
        const double2 ws = expipi(2.0 * nt / n);
#pragma unroll
        for (int jj = 0; jj < kHalfPerThread; jj++) {
            const int p = tid + jj * nt;
            if (p < h) {
                const double2 t = cmul(buf[pidx(p)], wp);
                buf[pidx(p)] = cadd(A[jj], t);
                buf[pidx(p + h)] = csub(A[jj], t);
            }
            wp = cmul(wp, ws);
        }
        __syncthreads();
    }

    // bins b = 0..n, split over NG groups of the residue classes for small rings
    const int nb = n + 1;
    const int NG = nb >= nt ? 1 : nt / nb;
    // e^{-i pi bin/n} and e^{-i pi bin/J}: with NG = 1 a thread's bins are
    // tid + j nt, stepped by products; with NG > 1 each thread has one bin
    const int bin0 = tid % nb;
    double2 qn = expipi(-(double)bin0 / n), qJ = s ? expipi(-(double)bin0 / J) : make_double2(1.0, 0.0);
    const double2 sn = expipi(-(double)nt / n), sJ = s ? expipi(-(double)nt / J) : make_double2(1.0, 0.0);
    for (int u = tid; u < NG * nb; u += nt) {
        const int g = u / nb, bin = u % nb;
        const double2 Zb = cconj(buf[pidx(bin == n ? 0 : bin)]);
        const double2 Znb = cconj(buf[pidx(bin == 0 ? 0 : n - bin)]);
        // F_b = (Z_b + conj Z_{n-b})/2 - (i/2) e^{-2 pi i b/J} (Z_b - conj Z_{n-b})
        const double2 e = cadd(Zb, cconj(Znb));
        const double2 d = cmul(csub(Zb, cconj(Znb)), qn);
        double2 F = make_double2(0.5 * (e.x + d.y), 0.5 * (e.y - d.x));
        double2 Gb = s ? cmul(F, qJ) : F;
        qn = cmul(qn, sn);
        qJ = cmul(qJ, sJ);
        // class 1: m = bin + jJ (j >= 0)
        for (long long j = g;; j += NG) {
            const long long m = bin + j * J;
            if (m > L) break;
            double2 v = (s & j & 1) ? make_double2(-Gb.x, -Gb.y) : Gb;
            if (m == 0) v = make_double2(v.x, 0.0);
            else v = make_double2(a.wpos * v.x, a.wpos * v.y);
            yr[(size_t)m * qstride] = v;
        }
        // class 2: m = jJ - bin (j >= 1); bins 0 and n are covered by class 1
        if (bin != 0 && bin != n) {
            for (long long j = (g == 0 ? NG : g);; j += NG) {
                const long long m = j * J - bin;
                if (m > L) break;
                double2 v = cconj(Gb);
                if (s & j & 1) v = make_double2(-v.x, -v.y);
                yr[(size_t)m * qstride] = make_double2(a.wpos * v.x, a.wpos * v.y);
            }
        }
    }
}

template <int T>
static hipError_t launch_analysis_classes(const sht_plan_s *p, RingArgs a, int nmaps, hipStream_t stream) {
    const void *fn[3] = {(const void *)k_ring_analysis<T, 1>, (const void *)k_ring_analysis<T, 2>,
                         (const void *)k_ring_analysis<T, 4>};
    for (const void *f : fn) {
        hipError_t ea = allow_dynamic_lds(f, 160 * 1024);
        if (ea != hipSuccess) return ea;
    }
    for (const auto &rc : p->classes) {
        a.rings = rc.d_rings;
        a.count = (int)rc.rings.size();
        a.fft_entries = rc.lds_entries + rc.lds_entries / 16;
        a.mpw = ring_maps_per_wg(rc.lds_entries, nmaps);
        long long grid = ((long long)a.count * nmaps / a.mpw + 63) / 64 * 64;
        size_t lds = (size_t)a.mpw * a.fft_entries * sizeof(double2);
        switch (a.mpw) {
            case 1: hipLaunchKernelGGL((k_ring_analysis<T, 1>), dim3((unsigned)grid), dim3(T), lds, stream, a); break;
            case 2: hipLaunchKernelGGL((k_ring_analysis<T, 2>), dim3((unsigned)grid), dim3(T), lds, stream, a); break;
            default: hipLaunchKernelGGL((k_ring_analysis<T, 4>), dim3((unsigned)grid), dim3(T), lds, stream, a); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_ring_analysis(const sht_plan_s *p, int nmaps, const double *map, double *ybar,
                                double wpos, hipStream_t stream) {
    RingArgs a;
    a.ring_J = p->d_ring_J;
    a.ring_s = p->d_ring_s;
    a.ring_M = p->d_ring_M;
    a.ring_off = p->d_ring_off;
    a.ring_bs_off = p->d_ring_bs_off;
    a.tw = reinterpret_cast<const double2 *>(p->d_tw);
    a.tw_log = p->tw_log;
    a.bs_table = reinterpret_cast<const double2 *>(p->d_bs_table);
    a.chirp = reinterpret_cast<const double2 *>(p->d_chirp);
    a.ring_chirp_off = p->d_ring_chirp_off;
    a.q = nullptr;
    a.map = nullptr;
    a.map_in = map;
    a.ybar = reinterpret_cast<double2 *>(ybar);
    a.wpos = wpos;
    a.L = p->L;
    a.nrings = p->nrings;
    a.nmaps = nmaps;
    a.npix = 12LL * p->nside * p->nside;
    a.stage = 0;
    switch (p->ring_threads) {
        case 256: return launch_analysis_classes<256>(p, a, nmaps, stream);
        case 512: return launch_analysis_classes<512>(p, a, nmaps, stream);
        default: return launch_analysis_classes<1024>(p, a, nmaps, stream);
    }
}

}  // namespace sht
