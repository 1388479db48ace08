// The fused substep kernels that also leave the restricted node copies of
// their output, in binary32 storage: the first two substeps of an RK3 step, in a
// translation unit of their own.
#include "octohydro_kernels.h"

namespace octohydro {

hipError_t launch_step_f32_restrict(const StepArgs& a, int blocks, StepShape sh,
                                       hipStream_t st) {
  return launch_step_t<float, STEP_RESTRICT>(a, blocks, sh, st);
}

}  // namespace octohydro
