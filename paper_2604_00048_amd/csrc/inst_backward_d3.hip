// Instantiations of the two-sweep kernels: backward, order d = 3.
#include "whs_two_sweep.h"

namespace whs {
hipError_t run_backward_d3(const LaunchDesc& L, hipStream_t stream) { return run_mode_d<3, Mode::Backward>(L, stream); }
}  // namespace whs
