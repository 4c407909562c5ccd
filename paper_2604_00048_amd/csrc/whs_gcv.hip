// GCV weight selection: launches of the grid-search kernel.
#include <hip/hip_runtime.h>

#include "whs_gcv.h"
#include "whs_kernels.h"

namespace whs {

// steps per loaded tile, and the number of grid values that share one pass
// over the inputs (the most whose recurrences fit in registers without spills:
// 21 grid values are three passes at order 1 or 2)
constexpr int gcv_tile(int) { return 8; }
constexpr int gcv_group(int D) { return D <= 2 ? 7 : (D == 3 ? 3 : 2); }

template <int D, typename TS>
static hipError_t gcv_t(const GcvLaunch& L, hipStream_t stream) {
  GcvArgs a;
  a.P = L.P;
  a.T = L.T;
  a.S = L.S;
  constexpr int B = gcv_tile(D);
  a.nt = (L.T + B - 1) / B;
  a.n_grid = L.n_grid;
  a.w = L.w;
  a.x = L.x;
  a.grid = L.grid;
  a.lam_best = L.lam_best;
  a.scores = L.scores;
  a.info = L.info;
  const int threads = 256;
  const int64_t blocks = (L.P + threads - 1) / threads;
  hipLaunchKernelGGL((k_gcv<D, B, TS, gcv_group(D)>), dim3((unsigned)blocks), dim3(threads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_gcv(const GcvLaunch& L, hipStream_t stream) {
  switch (L.D) {
    case 1: return L.f64 ? gcv_t<1, double>(L, stream) : gcv_t<1, float>(L, stream);
    case 2: return L.f64 ? gcv_t<2, double>(L, stream) : gcv_t<2, float>(L, stream);
    case 3: return L.f64 ? gcv_t<3, double>(L, stream) : gcv_t<3, float>(L, stream);
    case 4: return L.f64 ? gcv_t<4, double>(L, stream) : gcv_t<4, float>(L, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace whs
