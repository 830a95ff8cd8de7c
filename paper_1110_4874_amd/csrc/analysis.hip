// Element-wise steps of the quadrature analysis (Sec. 2.2, the quadrature
// rule a = sum_j w_j f_j Y*_lm(j) with the equal pixel weight 4 pi / Npix of
// the HEALPix grid) and of its Jacobi refinement a <- a + w Y^dagger (f - Y a):
// the Legendre and ring stages are the synthesis and adjoint kernels.
#include "internal.h"

namespace sht {

constexpr int kAxThreads = 256;

// y[i] = alpha x[i] + beta y[i] over n doubles (beta = 0 ignores y's contents).
__global__ __launch_bounds__(kAxThreads) void k_axpby(double *__restrict__ y, const double *__restrict__ x,
                                                      double alpha, double beta, long long n) {
    const long long i = (long long)blockIdx.x * kAxThreads + threadIdx.x;
    if (i >= n) return;
    y[i] = beta == 0.0 ? alpha * x[i] : __builtin_fma(alpha, x[i], beta * y[i]);
}

hipError_t launch_axpby(double *y, const double *x, double alpha, double beta, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + kAxThreads - 1) / kAxThreads)), dim3(kAxThreads), 0, st, y, x,
                       alpha, beta, n);
    return hipGetLastError();
}

}  // namespace sht
