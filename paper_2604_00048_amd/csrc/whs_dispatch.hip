// Dispatch of the two-sweep kernels over the difference order, and sizes.
#include <hip/hip_runtime.h>

#include "whs_two_sweep.h"

namespace whs {

hipError_t run_solve_d1(const LaunchDesc&, hipStream_t);
hipError_t run_solve_d2(const LaunchDesc&, hipStream_t);
hipError_t run_solve_d3(const LaunchDesc&, hipStream_t);
hipError_t run_solve_d4(const LaunchDesc&, hipStream_t);
hipError_t run_backward_d1(const LaunchDesc&, hipStream_t);
hipError_t run_backward_d2(const LaunchDesc&, hipStream_t);
hipError_t run_backward_d3(const LaunchDesc&, hipStream_t);
hipError_t run_backward_d4(const LaunchDesc&, hipStream_t);
hipError_t run_solve_tab_d1(const LaunchDesc&, hipStream_t);
hipError_t run_solve_tab_d2(const LaunchDesc&, hipStream_t);
hipError_t run_solve_tab_d3(const LaunchDesc&, hipStream_t);
hipError_t run_solve_tab_d4(const LaunchDesc&, hipStream_t);
hipError_t run_backward_tab_d1(const LaunchDesc&, hipStream_t);
hipError_t run_backward_tab_d2(const LaunchDesc&, hipStream_t);
hipError_t run_backward_tab_d3(const LaunchDesc&, hipStream_t);
hipError_t run_backward_tab_d4(const LaunchDesc&, hipStream_t);

size_t checkpoint_bytes(int64_t P, int S, int T, int D, int C) {
  // the largest checkpoint area any call with this descriptor can use:
  // the fast groupings (solve and adjoint), the generic one (given factor)
  // and the uneven-time one are all covered
  const int64_t nb = (P + S - 1) / S;
  size_t mx = 0;
  // generic, then the fast solve and adjoint for either storage type and weight kind
  for (int variant = 0; variant < 9; ++variant) {
    const bool fast = variant > 0, bwd = variant > 4, f64 = (variant - 1) & 1, perdiff = ((variant - 1) >> 1) & 1;
    for (int rem = C; rem > 0;) {
      const int g = next_group(rem, fast, D, bwd, f64, perdiff);
      size_t b = 0;
      switch (D) {
        case 1: b = ck_bytes_d<1>(nb, S, T, g); break;
        case 2: b = ck_bytes_d<2>(nb, S, T, g); break;
        case 3: b = ck_bytes_d<3>(nb, S, T, g); break;
        case 4: b = ck_bytes_d<4>(nb, S, T, g); break;
        default: return 0;
      }
      if (b > mx) mx = b;
      rem -= g;
    }
  }
  // the uneven-time groupings (fast path only): the solve's, and the adjoint's
  // for either storage type and weight kind
  for (int variant = 0; variant < 5; ++variant) {
    const bool bwd = variant > 0, f64 = variant > 2, perdiff = variant % 2 == 1;
    for (int rem = C; rem > 0;) {
      const int g = next_group_tab(rem, bwd, D, f64, perdiff);
      size_t b = 0;
      switch (D) {
        case 1: b = ck_bytes_tab_d<1>(nb, S, T, g); break;
        case 2: b = ck_bytes_tab_d<2>(nb, S, T, g); break;
        case 3: b = ck_bytes_tab_d<3>(nb, S, T, g); break;
        case 4: b = ck_bytes_tab_d<4>(nb, S, T, g); break;
        default: return 0;
      }
      if (b > mx) mx = b;
      rem -= g;
    }
  }
  return mx;
}

hipError_t launch_solve(const LaunchDesc& L, hipStream_t stream) {
  if (chunk_path(L)) return launch_chunk(L, false, stream);
  if (L.coef) {
    switch (L.D) {
      case 1: return run_solve_tab_d1(L, stream);
      case 2: return run_solve_tab_d2(L, stream);
      case 3: return run_solve_tab_d3(L, stream);
      case 4: return run_solve_tab_d4(L, stream);
      default: return hipErrorInvalidValue;
    }
  }
  switch (L.D) {
    case 1: return run_solve_d1(L, stream);
    case 2: return run_solve_d2(L, stream);
    case 3: return run_solve_d3(L, stream);
    case 4: return run_solve_d4(L, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_backward(const LaunchDesc& L, hipStream_t stream) {
  if (chunk_path(L)) return launch_chunk(L, true, stream);
  if (L.coef) {
    switch (L.D) {
      case 1: return run_backward_tab_d1(L, stream);
      case 2: return run_backward_tab_d2(L, stream);
      case 3: return run_backward_tab_d3(L, stream);
      case 4: return run_backward_tab_d4(L, stream);
      default: return hipErrorInvalidValue;
    }
  }
  switch (L.D) {
    case 1: return run_backward_d1(L, stream);
    case 2: return run_backward_d2(L, stream);
    case 3: return run_backward_d3(L, stream);
    case 4: return run_backward_d4(L, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace whs
