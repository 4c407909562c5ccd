// Internal launch interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace whs {

struct LaunchDesc {
  int64_t P;
  int T, D, C, S;
  bool f64;        // storage type of x, z, g, lambda and grads
  bool perdiff;    // lambda per difference row (else one scalar per series)
  const uint8_t* w;
  const void* lam;
  const double* fac;  // whs_factor output, or the factor to write (whs_factor)
  const void* rhs;    // x (solve) or g (backward)
  const void* zin;    // z (backward)
  void* out;          // z (solve) or grad_x (backward)
  void* glam;         // grad_lambda (backward)
  int32_t* info;
  double* ws;         // checkpoint workspace
  const double* coef = nullptr;  // rows of D on uneven sample times, (T-D) x (D+1); null: daily grid
  bool wbits = false;            // w one bit per series (S a multiple of 64, fused path only)
};

size_t checkpoint_bytes(int64_t P, int S, int T, int D, int C);
hipError_t launch_solve(const LaunchDesc& L, hipStream_t stream);
hipError_t launch_backward(const LaunchDesc& L, hipStream_t stream);
hipError_t launch_factor(const LaunchDesc& L, hipStream_t stream);
// (P, L) series-contiguous <-> (ceil(P/64), L, 64) interleaved, elements of 1, 4 or 8 bytes
hipError_t launch_interleave(const void* src, void* dst, int64_t P, int64_t L, int elem_bytes, bool to_interleaved,
                             hipStream_t stream);
// whether launch_interleave takes (P, L') with L' <= L, for elements of at most
// elem_bytes (4 or 8) and any alignment
bool interleave_fits(int64_t P, int64_t L, int elem_bytes);
// coefficient table of D from sample times: coef[k][j] = d! / prod_{m != j} (t[k+j] - t[k+m])
hipError_t launch_diff_coef(const double* times, int T, int D, double* coef, hipStream_t stream);

}  // namespace whs

namespace whs {

struct GcvLaunch {
  int64_t P;
  int T, D, S, n_grid;
  bool f64;
  const uint8_t* w;
  const void* x;
  const double* grid;
  void* lam_best;
  double* scores;
  int32_t* info;
};

hipError_t launch_gcv(const GcvLaunch& L, hipStream_t stream);

}  // namespace whs

namespace whs {

// posterior variance: L.out receives diag(Omega^{-1}) in the series layout
size_t var_checkpoint_bytes(int64_t P, int S, int T, int D);
hipError_t launch_var(const LaunchDesc& L, hipStream_t stream);

}  // namespace whs

namespace whs {

// several lanes per series (interleave 1, one band, order <= 2): see whs_chunk.hip
bool chunk_path(const LaunchDesc& L);
hipError_t launch_chunk(const LaunchDesc& L, bool bwd, hipStream_t stream);

}  // namespace whs
