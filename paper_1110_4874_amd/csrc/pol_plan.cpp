// Host tables of the polarized synthesis near the poles.
//
// The Discussion of the Wavemoth paper reduces the transform of a polarized
// map to scalar transforms (the cited reductions write the spin-2 harmonics
// through derivatives of scalar ones).  That reduction divides by
// sin^2(theta), so on the rings nearest the poles it loses ~eps / sin^2
// against the map's scale; there the spin-2 functions are evaluated
// directly instead, by the Wigner-d three-term recurrence in l started from
// Goldberg's closed form at l0 = max(m, 2):
//   _s lambda_{l0,m} = sgn K(m, s) sin^{2 l0 - c}(theta/2) cos^c(theta/2),
//   c = 2 r + s - m, r = max(0, m - s),
//   K = sqrt((2 l0 + 1)/(4 pi)) sqrt((l0+m)!(l0-m)!/((l0+s)!(l0-s)!))
//       C(l0 - s, r) C(l0 + s, r + s - m),
//   sgn = (-1)^(m + l0 - r - s).
// Everything here is exact rationals carried in double-double arithmetic.
#include <cmath>

#include "ddmath.h"
#include "internal.h"

namespace sht {

namespace {

dd ddv(double x) { return {x, 0.0}; }

// 2^e-normalised product: mant in [0.5, 1) (or 0) times 2^e
void renorm(dd &mant, long &e) {
    if (mant.h == 0.0) return;
    int ex;
    std::frexp(mant.h, &ex);
    mant.h = std::ldexp(mant.h, -ex);
    mant.l = std::ldexp(mant.l, -ex);
    e += ex;
}

}  // namespace

int build_pol_tables(sht_plan_s *p) {
    const int L = p->L, N = p->nside;
    // threshold: the reduction's error grows like eps sqrt(L) / sin^2(theta)
    // relative to the map; below sin(theta) = 0.1 sqrt((L+1)/4096) the
    // direct recurrence takes over (about 1e-13 at the threshold)
    const double s_pol = 0.1 * std::sqrt((double)(L + 1) / 4096.0);
    p->pol_ring.clear();
    p->pol_n = 0;
    for (int k = 0; k < p->n_north; k++) {
        // ring i = k + 1: z = num/den exactly (HEALPix RING scheme)
        const long i = k + 1;
        double num, den;
        if (i < N) {
            num = 3.0 * N * N - (double)i * i;
            den = 3.0 * N * N;
        } else {
            num = 4.0 * N - 2.0 * i;
            den = 3.0 * N;
        }
        // 1 - z = (den - num)/den, 1 + z = (den + num)/den, all exact integers
        const dd z = dd_div(ddv(num), ddv(den));
        const dd sh = dd_sqrt(dd_div(ddv(den - num), ddv(2.0 * den)));
        const dd ch = dd_sqrt(dd_div(ddv(den + num), ddv(2.0 * den)));
        const double sth = 2.0 * sh.h * ch.h;
        if (sth >= s_pol) break;
        p->pol_ring.insert(p->pol_ring.end(), {z.h, z.l, sh.h, sh.l, ch.h, ch.l});
        p->pol_n++;
    }
    p->pol_K.assign((size_t)(L + 1) * 2 * 4, 0.0);
    const dd four_pi = dd_mul(ddv(4.0), dd{3.141592653589793, 1.2246467991473532e-16});
    for (int m = 0; m <= L; m++)
        for (int si = 0; si < 2; si++) {
            const int s = si == 0 ? 2 : -2;
            const int l0 = m > 2 ? m : 2;
            const int r = m - s > 0 ? m - s : 0;
            dd mant = dd_sqrt(dd_div(ddv(2.0 * l0 + 1), four_pi));
            long e = 0;
            renorm(mant, e);
            if (l0 == m) {
                // sqrt(C(2m, m + s)) = prod_{j=1}^{m-s} sqrt((m + s + j)/j)
                for (int j = 1; j <= m - s; j++) {
                    mant = dd_mul(mant, dd_sqrt(dd_div(ddv((double)(m + s + j)), ddv((double)j))));
                    renorm(mant, e);
                }
            } else {
                // l0 = 2 > m: small factorials, exact in double
                double f[8] = {1, 1, 2, 6, 24, 120, 720, 5040};
                const double c1 = f[l0 - s] / (f[r] * f[l0 - s - r]);
                const double c2 = f[l0 + s] / (f[r + s - m] * f[l0 + s - (r + s - m)]);
                mant = dd_mul(mant, dd_sqrt(dd_div(ddv(f[l0 + m] * f[l0 - m]), ddv(f[l0 + s] * f[l0 - s]))));
                mant = dd_mul(mant, ddv(c1 * c2));
                renorm(mant, e);
            }
            if (((m + l0 - r - s) % 2 + 2) % 2) mant = dd_neg(mant);
            double *o = &p->pol_K[((size_t)m * 2 + si) * 4];
            o[0] = mant.h;
            o[1] = mant.l;
            o[2] = (double)e;
        }
    return SHT_OK;
}

// Host evaluation of _s lambda_lm at polar ring k (the GPU's recurrence and
// start, in the same double-double arithmetic): out[l - m], l = m .. L - 1.
int pol_column_host(const sht_plan_s *p, int m, int s, int k, double *out) {
    const int L = p->L, Lp = L - 1;
    if (m < 0 || m > Lp || (s != 2 && s != -2) || k < 0 || k >= p->pol_n) return SHT_EINVAL;
    for (int l = m; l <= Lp; l++) out[l - m] = 0.0;
    const int si = s == 2 ? 0 : 1;
    const int l0 = m > 2 ? m : 2;
    const int r = m - s > 0 ? m - s : 0;
    const int pc = 2 * r + s - m, ps = 2 * l0 - pc;
    const double *rg = &p->pol_ring[(size_t)k * 6];
    const dd z = {rg[0], rg[1]}, sh = {rg[2], rg[3]}, ch = {rg[4], rg[5]};
    const double *Kp = &p->pol_K[((size_t)m * 2 + si) * 4];
    dd mant = {Kp[0], Kp[1]};
    long e = (long)Kp[2];
    for (int j = 0; j < pc; j++) {
        mant = dd_mul(mant, ch);
        renorm(mant, e);
    }
    for (int j = 0; j < ps; j++) {
        mant = dd_mul(mant, sh);
        renorm(mant, e);
    }
    const double mm = (double)m * m;
    auto Asq = [&](double ll) {
        const double q = ll + 1.0;
        return dd_div(ddv((2.0 * ll + 3.0) * (2.0 * ll + 1.0) * q * q), ddv((q * q - mm) * (q * q - 4.0)));
    };
    dd p0 = {0.0, 0.0}, p1 = mant;
    for (int l = l0; l <= Lp; l++) {
        out[l - m] = e < -4000 ? 0.0 : std::ldexp(p1.h, (int)e);
        if (l == Lp) break;
        const dd A = dd_sqrt(Asq((double)l));
        const dd Bc = (l == l0) ? dd{0.0, 0.0} : dd_div(A, dd_sqrt(Asq((double)l - 1.0)));
        const dd C = dd_div(ddv((double)m * s), ddv((double)l * (l + 1.0)));
        const dd nx = dd_sub(dd_mul(dd_mul(A, dd_add(z, C)), p1), dd_mul(Bc, p0));
        p0 = p1;
        p1 = nx;
        if (std::fabs(p1.h) > 0x1p300) {
            p0 = {std::ldexp(p0.h, -300), std::ldexp(p0.l, -300)};
            p1 = {std::ldexp(p1.h, -300), std::ldexp(p1.l, -300)};
            e += 300;
        }
    }
    return SHT_OK;
}

}  // namespace sht
