// Instantiations of the two-sweep kernels: solve, order d = 1.
#include "whs_two_sweep.h"

namespace whs {
hipError_t run_solve_d1(const LaunchDesc& L, hipStream_t stream) { return run_mode_d<1, Mode::Solve>(L, stream); }
}  // namespace whs
