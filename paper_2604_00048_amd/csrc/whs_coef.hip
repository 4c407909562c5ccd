// Rows of the difference operator on uneven sample times (Sec. II): the
// order-d discrete derivative is d! times the divided difference over d+1
// consecutive sample times,
//   (D v)_k = sum_j c[k][j] v_{k+j},   c[k][j] = d! / prod_{m != j} (t_{k+j} - t_{k+m}).
// One thread per row.  Rows whose times are not strictly increasing (or not
// finite) are NaN, so every solve that uses them fails visibly.
#include <hip/hip_runtime.h>

#include "whs_kernels.h"

namespace whs {

__global__ __launch_bounds__(256) void k_diff_coef(const double* __restrict__ times, int T, int D,
                                                   double* __restrict__ coef) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T - D) return;
  double tt[5];
  for (int j = 0; j <= D; ++j) tt[j] = times[k + j];
  bool ok = true;
  for (int j = 0; j < D; ++j) ok = ok && (tt[j + 1] > tt[j]) && (tt[j + 1] - tt[j] < __builtin_huge_val());
  double fact = 1.0;
  for (int i = 2; i <= D; ++i) fact *= (double)i;
  for (int j = 0; j <= D; ++j) {
    double den = 1.0;
    for (int m = 0; m <= D; ++m)
      if (m != j) den *= tt[j] - tt[m];
    coef[(int64_t)k * (D + 1) + j] = ok ? fact / den : __builtin_nan("");
  }
}

hipError_t launch_diff_coef(const double* times, int T, int D, double* coef, hipStream_t stream) {
  const int rows = T - D;
  const int threads = 256;
  hipLaunchKernelGGL(k_diff_coef, dim3((unsigned)((rows + threads - 1) / threads)), dim3(threads), 0, stream, times,
                     T, D, coef);
  return hipGetLastError();
}

}  // namespace whs
