// The fused substep kernel k_step in binary64: its instantiations for
// every field count and register budget live in this translation unit.
#include "octohydro_kernels.h"

namespace octohydro {

hipError_t launch_step_f64(const StepArgs& a, int blocks, StepShape sh, hipStream_t st) {
  return launch_step_t<double, STEP_PLAIN>(a, blocks, sh, st);
}

}  // namespace octohydro
