// Instantiations of the two-sweep kernels: backward, order d = 1.
#include "whs_two_sweep.h"

namespace whs {
hipError_t run_backward_d1(const LaunchDesc& L, hipStream_t stream) { return run_mode_d<1, Mode::Backward>(L, stream); }
}  // namespace whs
