// Instantiations of the two-sweep kernels: solve, order d = 3.
#include "whs_two_sweep.h"

namespace whs {
hipError_t run_solve_d3(const LaunchDesc& L, hipStream_t stream) { return run_mode_d<3, Mode::Solve>(L, stream); }
}  // namespace whs
