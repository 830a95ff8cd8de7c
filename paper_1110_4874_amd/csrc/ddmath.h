// Double-double arithmetic for the compensated recurrences near the poles
// (error-free transformations: Knuth's two-sum, Dekker's fast two-sum, and
// products with the FMA's exact remainder).  FMA contraction is switched off
// so that every sum is formed exactly as written.
#pragma once
#include <hip/hip_runtime.h>

namespace sht {

struct dd {
    double h, l;
};

#pragma clang fp contract(off)
__host__ __device__ __forceinline__ dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__host__ __device__ __forceinline__ dd fast_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}
__host__ __device__ __forceinline__ dd dd_mul(dd a, dd b) {
    double p = a.h * b.h;
    double e = __builtin_fma(a.h, b.h, -p);
    e = __builtin_fma(a.h, b.l, e);
    e = __builtin_fma(a.l, b.h, e);
    return fast_two_sum(p, e);
}
__host__ __device__ __forceinline__ dd dd_add(dd a, dd b) {
    dd s = two_sum(a.h, b.h);
    double e = s.l + (a.l + b.l);
    return fast_two_sum(s.h, e);
}
__host__ __device__ __forceinline__ dd dd_neg(dd a) { return {-a.h, -a.l}; }
__host__ __device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
// a / b: three quotient digits (Newton-free long division, each digit a
// correctly rounded double quotient of the running remainder)
__host__ __device__ __forceinline__ dd dd_div(dd a, dd b) {
    const double q1 = a.h / b.h;
    dd r = dd_sub(a, dd_mul(b, {q1, 0.0}));
    const double q2 = r.h / b.h;
    r = dd_sub(r, dd_mul(b, {q2, 0.0}));
    const double q3 = r.h / b.h;
    return dd_add(fast_two_sum(q1, q2), {q3, 0.0});
}
// sqrt(a), a > 0: one Newton correction of the double root, q + (a - q^2)/(2q)
__host__ __device__ __forceinline__ dd dd_sqrt(dd a) {
    const double q = sqrt(a.h);
    const dd r = dd_sub(a, dd_mul({q, 0.0}, {q, 0.0}));
    return fast_two_sum(q, r.h / (2.0 * q));
}
#pragma clang fp contract(on)

}  // namespace sht
