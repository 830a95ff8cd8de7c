// Polarized (spin-2) synthesis as scalar transforms, for gfx950.
//
// The Discussion of the Wavemoth paper notes that the transform of a
// polarized map reduces to three scalar transforms (citing the reductions
// through spin-raising operators), which also amortises the streaming of
// the precomputed data.  With a_{+-2,lm} = -(E_lm +- i B_lm) and
// Q +- iU = sum a_{+-2,lm} _{+-2}Y_lm, the spin-2 functions follow from the
// scalar ones by two spin raisings; with N_l = sqrt((l-2)!/(l+2)!),
// c = cos(theta), s = sin(theta):
//   F1 = (_2 lambda + _-2 lambda)/2 = N_l [2 (m^2 lambda - c s lambda')/s^2 - l(l+1) lambda]
//   F2 = (_2 lambda - _-2 lambda)/2 = N_l 2 m (c lambda - s lambda')/s^2
// and s lambda'_lm = l e_{l+1} lambda_{l+1} - (l+1) e_l lambda_{l-1},
// e_l = sqrt((l^2 - m^2)/(4 l^2 - 1)).  So per mode (E, B) three scalar
// coefficient sets, of band limit L = L_pol + 1,
//   S0: N_l a_l,  S1: l(l+1) N_l a_l,
//   S2: (l-1) e_l N_{l-1} a_{l-1} - (l+2) e_{l+1} N_{l+1} a_{l+1},
// run through the scalar Legendre phase as six maps per polarized map (one
// pass over the plan's data for all of them), and per ring and order
//   F1 = 2 (m^2 S0 - c S2)/s^2 - S1,   F2 = 2 m (c S0 - S2)/s^2,
//   Q_m = -(F1[E] + i F2[B]),   U_m = -(F1[B] - i F2[E]),
// then the scalar ring stage on 2 maps per polarized map.
//
// The division by s^2 costs ~eps / s^2 of the map's scale near the poles;
// on the rings with s below the plan's threshold the spin-2 functions are
// evaluated directly instead: the Wigner-d three-term recurrence in l,
//   _s lambda_{l+1} = A_l (c + m s/(l(l+1))) _s lambda_l - (A_l / A_{l-1}) _s lambda_{l-1},
//   A_l = sqrt((2l+3)(2l+1)(l+1)^2 / (((l+1)^2 - m^2)((l+1)^2 - s^2))),
// in double-double arithmetic (the z-based recurrence loses ~l eps / s in
// FP64) from Goldberg's closed form at l0 = max(m, 2), with the plan's
// per-(m, s) start factors; one wave per (m, 64 polar rings), both
// hemispheres from one recurrence (_s lambda(pi - theta) =
// (-1)^(l+m) _{-s} lambda(theta)).
#include "ddmath.h"
#include "internal.h"

namespace sht {

namespace {

__device__ __forceinline__ double2 ld2(const double *p) { return *reinterpret_cast<const double2 *>(p); }

}  // namespace

// ---- coefficient sets -------------------------------------------------------
// One workgroup per order m; E, B: [nalm(L-1)][n] complex; out: [nalm(L)][6n]
// complex, map 6b + {0, 1, 2} = S0, S1, S2 of E_b, 6b + {3, 4, 5} of B_b.
__global__ __launch_bounds__(256) void k_pol_prep(const double *__restrict__ E, const double *__restrict__ B,
                                                  double *__restrict__ out, int L, int n) {
    const int m = blockIdx.x;
    const int Lp = L - 1;
    const size_t offo = (size_t)m * (2 * L + 3 - m) / 2;
    const size_t offi = (size_t)m * (2 * Lp + 3 - m) / 2;  // valid for m <= Lp
    auto coef = [&](const double *A, int l, int b) -> double2 {
        // N_l a_lm for 2 <= l <= Lp, l >= m; Im a_l0 ignored
        if (l < 2 || l < m || l > Lp) return make_double2(0.0, 0.0);
        const double2 a = ld2(A + 2 * ((offi + l - m) * n + b));
        const double nl = 1.0 / sqrt((double)(l - 1) * l * (double)(l + 1) * (l + 2));
        return make_double2(a.x * nl, m == 0 ? 0.0 : a.y * nl);
    };
    auto eps = [&](int l) -> double {
        return l > m ? sqrt(((double)l * l - (double)m * m) / (4.0 * l * l - 1.0)) : 0.0;
    };
    const int cnt = (L - m + 1) * n;
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const int l = m + e / n, b = e % n;
        const double el = eps(l), el1 = eps(l + 1);
        double2 *o = reinterpret_cast<double2 *>(out) + (offo + l - m) * 6 * n + 6 * b;
        for (int mode = 0; mode < 2; mode++) {
            const double *A = mode ? B : E;
            const double2 c = coef(A, l, b), cm1 = coef(A, l - 1, b), cp1 = coef(A, l + 1, b);
            const double w = (double)l * (l + 1);
            o[3 * mode + 0] = c;
            o[3 * mode + 1] = make_double2(w * c.x, w * c.y);
            const double f0 = (double)(l - 1) * el, f1 = (double)(l + 2) * el1;
            o[3 * mode + 2] = make_double2(f0 * cm1.x - f1 * cp1.x, f0 * cm1.y - f1 * cp1.y);
        }
    }
}

// ---- spin-2 combination -----------------------------------------------------
// One thread per (ring, m, polarized map): q6 [rings][L+1][6n] -> q2
// [rings][L+1][2n] (Q of map b at b, U at n + b).
__global__ __launch_bounds__(256) void k_pol_combine(const double *__restrict__ q6, double *__restrict__ q2,
                                                     const double *__restrict__ z2_hi,
                                                     const double *__restrict__ z2_lo, int L, int nrings,
                                                     int n_north, int n, long long total) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const int b = (int)(t % n);
    const long long rm = t / n;
    const int m = (int)(rm % (L + 1)), r = (int)(rm / (L + 1));
    const int k = r < n_north ? r : nrings - 1 - r;
    const double zz = z2_hi[k];
    const double c = r < n_north ? sqrt(zz) : -sqrt(zz);
    const double s2 = (1.0 - zz) - z2_lo[k];
    const double2 *S = reinterpret_cast<const double2 *>(q6) + (size_t)rm * 6 * n + 6 * b;
    const double mm = (double)m * m, inv = 1.0 / s2;
    double2 F1[2], F2[2];
    for (int mode = 0; mode < 2; mode++) {
        const double2 S0 = S[3 * mode], S1 = S[3 * mode + 1], S2 = S[3 * mode + 2];
        F1[mode] = make_double2(2.0 * (mm * S0.x - c * S2.x) * inv - S1.x, 2.0 * (mm * S0.y - c * S2.y) * inv - S1.y);
        F2[mode] = make_double2(2.0 * m * (c * S0.x - S2.x) * inv, 2.0 * m * (c * S0.y - S2.y) * inv);
    }
    // Q = -(F1[E] + i F2[B]),  U = -(F1[B] - i F2[E])
    double2 Q = make_double2(-F1[0].x + F2[1].y, -F1[0].y - F2[1].x);
    double2 U = make_double2(-F1[1].x - F2[0].y, -F1[1].y + F2[0].x);
    if (m == 0) Q.y = U.y = 0.0;  // real fields
    double2 *o = reinterpret_cast<double2 *>(q2) + (size_t)rm * 2 * n;
    o[b] = Q;
    o[n + b] = U;
}

// ---- polar caps: the spin-2 recurrence itself -------------------------------
struct PolArgs {
    const double *__restrict__ E;
    const double *__restrict__ B;
    const double *__restrict__ ring;  // [pol_n][6] z, sin(theta/2), cos(theta/2) (hi, lo)
    const double *__restrict__ K;     // [(L+1)*2][4]
    const int *__restrict__ grp_lo;   // scalar chain starts per (m, 64-ring group)
    double *__restrict__ q2;
    int L, nrings, pol_n, ng, ngp, n, map0;  // ng: the plan's 64-ring groups, ngp: polar groups
};

__device__ __forceinline__ double rdl(double x, int j) {  // lane j's x (j wave-uniform)
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffLL), j);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), j);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// mant * base^p with exponent tracking (mant kept in [0.5, 1) by powers of 2)
__device__ __forceinline__ void dd_pow_acc(dd &mant, int &e, dd base, int p) {
    int eb;
    const double bh = frexp(base.h, &eb);
    dd bm = {bh, ldexp(base.l, -eb)};
    int ex;
    for (; p > 0; p >>= 1) {
        if (p & 1) {
            mant = dd_mul(mant, bm);
            e += eb;
            const double h = frexp(mant.h, &ex);
            mant = {h, ldexp(mant.l, -ex)};
            e += ex;
        }
        bm = dd_mul(bm, bm);
        eb *= 2;
        const double h = frexp(bm.h, &ex);
        bm = {h, ldexp(bm.l, -ex)};
        eb += ex;
    }
}

template <int NB>
__global__ __launch_bounds__(64) void k_pol_polar(PolArgs a) {
    const int m = blockIdx.x / a.ngp, g = blockIdx.x % a.ngp;
    const int L = a.L, Lp = L - 1, lane = threadIdx.x;
    if (m > Lp) return;
    const int n0 = (L - m) / 2 + 1;
    const int lo = a.grp_lo[(size_t)m * a.ng + g];
    if (lo >= n0) return;  // every chain of this group stays below the cutoff: the combination wrote 0
    const int k = g * 64 + lane;
    const bool act = k < a.pol_n;
    const int kk = act ? k : a.pol_n - 1;
    const dd z = {a.ring[6 * kk], a.ring[6 * kk + 1]};
    const dd sh = {a.ring[6 * kk + 2], a.ring[6 * kk + 3]};
    const dd chh = {a.ring[6 * kk + 4], a.ring[6 * kk + 5]};
    const int l0 = m > 2 ? m : 2;
    // start values and exponents of s = +2 (index 0) and s = -2 (index 1)
    dd p0[2], p1[2];  // lambda_{l-1}, lambda_l (scaled by 2^-E)
    int Ex[2];
#pragma unroll
    for (int si = 0; si < 2; si++) {
        const int s = si == 0 ? 2 : -2;
        const int r = m - s > 0 ? m - s : 0;
        const int pc = 2 * r + s - m, ps = 2 * l0 - pc;
        const double *Kp = a.K + ((size_t)m * 2 + si) * 4;
        dd mant = {Kp[0], Kp[1]};
        int e = (int)Kp[2];
        dd_pow_acc(mant, e, chh, pc);
        dd_pow_acc(mant, e, sh, ps);
        p0[si] = {0.0, 0.0};
        p1[si] = mant;
        Ex[si] = e;
    }
    // accumulators per map: [parity of l - m][E F1, B F2, B F1, E F2] complex
    double acc[NB][2][4][2];
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int pp = 0; pp < 2; pp++)
#pragma unroll
            for (int q = 0; q < 4; q++) acc[b][pp][q][0] = acc[b][pp][q][1] = 0.0;
    const size_t offi = (size_t)m * (2 * Lp + 3 - m) / 2;
    const double mm = (double)m * m;
    for (int lb = l0; lb <= Lp; lb += 64) {
        // recurrence coefficients of steps l -> l + 1, l = lb + lane
        const int l = lb + lane;
        const double lp = l + 1.0;
        auto Asq = [&](double ll) {  // A_{ll}^2 as an exact ratio, ll = l
            const double q = ll + 1.0;
            return dd_div(dd{(2.0 * ll + 3.0) * (2.0 * ll + 1.0) * q * q, 0.0},
                          dd{(q * q - mm) * (q * q - 4.0), 0.0});
        };
        const dd A = dd_sqrt(Asq((double)l));
        const dd Bc = (l == l0) ? dd{0.0, 0.0} : dd_div(A, dd_sqrt(Asq((double)l - 1.0)));
        const dd C = dd_div(dd{2.0 * m, 0.0}, dd{(double)l * lp, 0.0});  // m s / (l(l+1)), s = +2
        const double Ah = A.h, Al = A.l, Bh = Bc.h, Bl = Bc.l, Ch = C.h, Cl = C.l;
        const int steps = min(64, Lp - lb + 1);
        for (int j = 0; j < steps; j++) {
            const int lc = lb + j;
            const int par = (lc - m) & 1;
            // accumulate l = lc
            const double fp = ldexp(p1[0].h, max(Ex[0], -4000)), fm = ldexp(p1[1].h, max(Ex[1], -4000));
            const double F1 = 0.5 * (fp + fm), F2 = 0.5 * (fp - fm);
            const double *Er = a.E + 2 * ((offi + lc - m) * a.n + a.map0);
            const double *Br = a.B + 2 * ((offi + lc - m) * a.n + a.map0);
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const double er = Er[2 * b], ei = m ? Er[2 * b + 1] : 0.0;
                const double br = Br[2 * b], bi = m ? Br[2 * b + 1] : 0.0;
                acc[b][par][0][0] = __builtin_fma(er, F1, acc[b][par][0][0]);
                acc[b][par][0][1] = __builtin_fma(ei, F1, acc[b][par][0][1]);
                acc[b][par][1][0] = __builtin_fma(br, F2, acc[b][par][1][0]);
                acc[b][par][1][1] = __builtin_fma(bi, F2, acc[b][par][1][1]);
                acc[b][par][2][0] = __builtin_fma(br, F1, acc[b][par][2][0]);
                acc[b][par][2][1] = __builtin_fma(bi, F1, acc[b][par][2][1]);
                acc[b][par][3][0] = __builtin_fma(er, F2, acc[b][par][3][0]);
                acc[b][par][3][1] = __builtin_fma(ei, F2, acc[b][par][3][1]);
            }
            if (lc == Lp) break;
            // advance to lc + 1
            const dd Aj = {rdl(Ah, j), rdl(Al, j)}, Bj = {rdl(Bh, j), rdl(Bl, j)}, Cj = {rdl(Ch, j), rdl(Cl, j)};
#pragma unroll
            for (int si = 0; si < 2; si++) {
                const dd w = dd_mul(Aj, dd_add(z, si == 0 ? Cj : dd_neg(Cj)));
                const dd nx = dd_sub(dd_mul(w, p1[si]), dd_mul(Bj, p0[si]));
                p0[si] = p1[si];
                p1[si] = nx;
                if (fabs(nx.h) > 0x1p300) {
                    p0[si] = {ldexp(p0[si].h, -300), ldexp(p0[si].l, -300)};
                    p1[si] = {ldexp(p1[si].h, -300), ldexp(p1[si].l, -300)};
                    Ex[si] += 300;
                }
            }
        }
    }
    if (!act) return;
    const int ks = a.nrings - 1 - k;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        // north: parity sums added; south: F1 -> (-1)^(l+m) F1, F2 -> -(-1)^(l+m) F2
        double s[2][4][2];
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int c = 0; c < 2; c++) {
                s[0][q][c] = acc[b][0][q][c] + acc[b][1][q][c];
                const double d = acc[b][0][q][c] - acc[b][1][q][c];
                s[1][q][c] = (q == 0 || q == 2) ? d : -d;
            }
#pragma unroll
        for (int h = 0; h < 2; h++) {
            // Q = -(sum E F1 + i sum B F2), U = -(sum B F1 - i sum E F2)
            double2 Q = make_double2(-s[h][0][0] + s[h][1][1], -s[h][0][1] - s[h][1][0]);
            double2 U = make_double2(-s[h][2][0] - s[h][3][1], -s[h][2][1] + s[h][3][0]);
            if (m == 0) Q.y = U.y = 0.0;
            const int ring = h == 0 ? k : ks;
            double2 *o = reinterpret_cast<double2 *>(a.q2) + ((size_t)ring * (L + 1) + m) * 2 * a.n;
            o[a.map0 + b] = Q;
            o[a.n + a.map0 + b] = U;
        }
    }
}

size_t pol_alm_bytes(const sht_plan_s *p, int nmaps) {
    return ((size_t)(p->L + 1) * (p->L + 2) / 2 * 6 * nmaps * 16 + 255) / 256 * 256;
}

hipError_t launch_pol_prep(const sht_plan_s *p, int nmaps, const double *E, const double *B, double *alm6,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_pol_prep, dim3((unsigned)(p->L + 1)), dim3(256), 0, st, E, B, alm6, p->L, nmaps);
    return hipGetLastError();
}

hipError_t launch_pol_combine(const sht_plan_s *p, int nmaps, const double *q6, double *q2, hipStream_t st) {
    const long long total = (long long)p->nrings * (p->L + 1) * nmaps;
    hipLaunchKernelGGL(k_pol_combine, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, q6, q2, p->d_z2_hi,
                       p->d_z2_lo, p->L, p->nrings, p->n_north, nmaps, total);
    return hipGetLastError();
}

hipError_t launch_pol_polar(const sht_plan_s *p, int nmaps, const double *E, const double *B, double *q2,
                            hipStream_t st) {
    if (p->pol_n == 0 || p->L < 3) return hipSuccess;
    PolArgs a;
    a.E = E;
    a.B = B;
    a.ring = p->d_pol_ring;
    a.K = p->d_pol_K;
    a.grp_lo = p->d_grp_lo;
    a.q2 = q2;
    a.L = p->L;
    a.nrings = p->nrings;
    a.pol_n = p->pol_n;
    a.n = nmaps;
    a.ng = p->n_north_pad / kLanes;
    a.ngp = (p->pol_n + 63) / 64;
    hipError_t e = hipSuccess;
    for (int b = 0; b < nmaps && e == hipSuccess;) {
        const int nb = nmaps - b >= 2 ? 2 : 1;
        a.map0 = b;
        const dim3 grid((unsigned)(p->L * a.ngp));  // orders 0 .. L-1 x polar groups
        if (nb == 2)
            hipLaunchKernelGGL(k_pol_polar<2>, grid, dim3(64), 0, st, a);
        else
            hipLaunchKernelGGL(k_pol_polar<1>, grid, dim3(64), 0, st, a);
        e = hipGetLastError();
        b += nb;
    }
    return e;
}

}  // namespace sht
