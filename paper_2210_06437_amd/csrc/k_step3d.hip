// The 3D-reconstruction step kernel k_step3d: its instantiations for every
// field count and both precisions live in this translation unit.
#include "octohydro_kernels3d.h"

namespace octohydro {

hipError_t launch_step3d(const StepArgs& a, int dtype, int blocks, const void* G, int wg,
                         hipStream_t st) {
  return dtype == HYDRO_F64
             ? launch_step3d_t<double>(a, blocks, static_cast<const double*>(G), wg, st)
             : launch_step3d_t<float>(a, blocks, static_cast<const float*>(G), wg, st);
}

}  // namespace octohydro
