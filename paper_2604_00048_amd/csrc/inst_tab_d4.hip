// Instantiations of the two-sweep kernels on uneven sample times: order d = 4.
#include "whs_two_sweep.h"

namespace whs {
hipError_t run_solve_tab_d4(const LaunchDesc& L, hipStream_t stream) { return run_mode_tab_d<4, Mode::Solve>(L, stream); }
hipError_t run_backward_tab_d4(const LaunchDesc& L, hipStream_t stream) {
  return run_mode_tab_d<4, Mode::Backward>(L, stream);
}
}  // namespace whs
