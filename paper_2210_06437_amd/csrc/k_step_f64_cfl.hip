// The fused substep kernels with the CFL epilogue in binary64: the last
// substep of a chained RK3 step, in a translation unit of their own.
#include "octohydro_kernels.h"

namespace octohydro {

hipError_t launch_step_f64_cfl(const StepArgs& a, int blocks, StepShape sh, hipStream_t st) {
  return launch_step_t<double, STEP_CFL>(a, blocks, sh, st);
}

}  // namespace octohydro
