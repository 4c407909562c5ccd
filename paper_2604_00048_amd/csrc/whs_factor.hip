// whs_factor kernel: the Cholesky factor of Omega in lower band storage.
#include <hip/hip_runtime.h>

#include "whs_kernels.h"
#include "whs_step.h"

namespace whs {

// ---------------------------------------------------------------------------
// whs_factor: sweep 1 only, writing the Cholesky factor (Alg. 1 output)
// F[i][t] = L[t+i, t] sqrt(Dp[t]) in lower band storage (Fig. 2).
// ---------------------------------------------------------------------------
template <int D, typename TS, bool PERDIFF>
__global__ __launch_bounds__(256) void k_factor(int64_t P, int T, int S, const uint8_t* w, const void* lam,
                                                double* fac, int32_t* info_out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t bidx = p / S;
  const int sl = static_cast<int>(p - bidx * S);
  const uint8_t* ws = w + (int64_t)bidx * T * S + sl;
  const TS* ls = PERDIFF ? static_cast<const TS*>(lam) + (int64_t)bidx * (T - D) * S + sl : nullptr;
  const double lam_s = PERDIFF ? 0.0 : to_f64(static_cast<const TS*>(lam)[p]);
  double* fs = fac + (int64_t)bidx * (D + 1) * T * S + sl;
  State<D, 1> st;
  st.zero();
  double sq[D + 1];  // sqrt(Dp[t-j])
#pragma unroll
  for (int j = 0; j <= D; ++j) sq[j] = 0.0;
  int info = 0, nobs = 0;
  for (int t = 0; t < T; ++t) {
    const bool obs = ws[(int64_t)t * S] != 0;
    nobs += obs;
    double lw[D + 1];
    const double lt = (t < T - D) ? (PERDIFF ? to_f64(ls[(int64_t)t * S]) : lam_s) : 0.0;
    lw[0] = lt;
#pragma unroll
    for (int m = 1; m <= D; ++m) lw[m] = st.lw[m];
    double om[D + 1], l[D + 1], dt, invdt;
    omega_row<D>(lw, obs ? 1.0 : 0.0, om);
    ldl_step<D, 1>(st, om, l, dt, invdt);
#pragma unroll
    for (int m = D; m >= 2; --m) st.lw[m] = st.lw[m - 1];
    st.lw[1] = lt;
    if (!pivot_ok(dt) && info == 0) info = t + 1;
    const double sd = __builtin_sqrt(dt);
    fs[((int64_t)0 * T + t) * S] = sd;
#pragma unroll
    for (int j = 1; j <= D; ++j)
      if (t - j >= 0) fs[((int64_t)j * T + (t - j)) * S] = l[j] * sq[j];
#pragma unroll
    for (int j = D; j >= 2; --j) sq[j] = sq[j - 1];
    sq[1] = sd;
  }
  // zero tail: F[i][t] with t + i >= T
#pragma unroll
  for (int i = 1; i <= D; ++i)
    for (int t = T - i; t < T; ++t)
      if (t >= 0) fs[((int64_t)i * T + t) * S] = 0.0;
  if (info == 0 && nobs < D) info = T;
  if (info != 0) {
    const double qnan = __builtin_nan("");
    for (int i = 0; i <= D; ++i)
      for (int t = 0; t < T; ++t) fs[((int64_t)i * T + t) * S] = qnan;
  }
  if (info_out) info_out[p] = info;
}

template <int D, typename TS, bool PERDIFF>
static hipError_t launch_factor_t(const LaunchDesc& L, hipStream_t stream) {
  const int threads = 256;
  const int64_t blocks = (L.P + threads - 1) / threads;
  hipLaunchKernelGGL((k_factor<D, TS, PERDIFF>), dim3((unsigned)blocks), dim3(threads), 0, stream, L.P, L.T, L.S,
                     L.w, L.lam, const_cast<double*>(L.fac), L.info);
  return hipGetLastError();
}

template <typename TS, bool PERDIFF>
static hipError_t launch_factor_k(const LaunchDesc& L, hipStream_t stream) {
  switch (L.D) {
    case 1: return launch_factor_t<1, TS, PERDIFF>(L, stream);
    case 2: return launch_factor_t<2, TS, PERDIFF>(L, stream);
    case 3: return launch_factor_t<3, TS, PERDIFF>(L, stream);
    case 4: return launch_factor_t<4, TS, PERDIFF>(L, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_factor(const LaunchDesc& L, hipStream_t stream) {
  if (L.f64) return L.perdiff ? launch_factor_k<double, true>(L, stream) : launch_factor_k<double, false>(L, stream);
  return L.perdiff ? launch_factor_k<float, true>(L, stream) : launch_factor_k<float, false>(L, stream);
}

}  // namespace whs
