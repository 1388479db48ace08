// The fused substep kernel k_step in binary32 storage (FP32-mixed): its instantiations for
// every field count and register budget live in this translation unit.
#include "octohydro_kernels.h"

namespace octohydro {

hipError_t launch_step_f32(const StepArgs& a, int blocks, StepShape sh, hipStream_t st) {
  return launch_step_t<float, STEP_PLAIN>(a, blocks, sh, st);
}

}  // namespace octohydro
