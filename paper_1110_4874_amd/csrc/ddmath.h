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

}  // namespace sht
