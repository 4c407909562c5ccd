// Posterior variance (diagonal of Omega^{-1}): launches of the variance kernel.
#include <hip/hip_runtime.h>

#include "whs_fast.h"
#include "whs_kernels.h"

namespace whs {

// tile depth: the reverse sweep keeps 1/Dp and the band of L per step, as GCV does
constexpr int var_tile(int D) { return D <= 2 ? 16 : 8; }

size_t var_checkpoint_bytes(int64_t P, int S, int T, int D) {
  const int64_t nb = (P + S - 1) / S;
  const int64_t nt = (T + var_tile(D) - 1) / var_tile(D);
  int nf = 0;
  switch (D) {
    case 1: nf = ck_fields<1, 1>(); break;
    case 2: nf = ck_fields<2, 1>(); break;
    case 3: nf = ck_fields<3, 1>(); break;
    case 4: nf = ck_fields<4, 1>(); break;
    default: return 0;
  }
  return (size_t)nb * nt * nf * S * sizeof(double);
}

template <int D, typename TS, bool PERDIFF>
static hipError_t var_t(const LaunchDesc& L, hipStream_t stream) {
  VarArgs a;
  a.P = L.P;
  a.T = L.T;
  a.S = L.S;
  constexpr int B = var_tile(D);
  a.nt = (L.T + B - 1) / B;
  a.w = L.w;
  a.lam = L.lam;
  a.var = L.out;
  a.info = L.info;
  a.ck = L.ws;
  const int threads = 256;
  const int64_t blocks = (L.P + threads - 1) / threads;
  hipLaunchKernelGGL((k_var<D, B, TS, PERDIFF>), dim3((unsigned)blocks), dim3(threads), 0, stream, a);
  return hipGetLastError();
}

template <int D>
static hipError_t var_d(const LaunchDesc& L, hipStream_t stream) {
  if (L.f64) return L.perdiff ? var_t<D, double, true>(L, stream) : var_t<D, double, false>(L, stream);
  return L.perdiff ? var_t<D, float, true>(L, stream) : var_t<D, float, false>(L, stream);
}

hipError_t launch_var(const LaunchDesc& L, hipStream_t stream) {
  switch (L.D) {
    case 1: return var_d<1>(L, stream);
    case 2: return var_d<2>(L, stream);
    case 3: return var_d<3>(L, stream);
    case 4: return var_d<4>(L, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace whs
