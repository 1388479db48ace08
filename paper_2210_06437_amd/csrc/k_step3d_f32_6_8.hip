// Instantiations of the 3D step kernel k_step3d, binary32 storage, 6 to 8
// fields: one of the units its instantiations are spread over so that they
// compile in parallel.
#include "octohydro_kernels3d.h"

namespace octohydro {

template hipError_t launch_step3d_one<float, 6>(const StepArgs&, int, const float*, int,
                                     hipStream_t);
template hipError_t launch_step3d_one<float, 7>(const StepArgs&, int, const float*, int,
                                     hipStream_t);
template hipError_t launch_step3d_one<float, 8>(const StepArgs&, int, const float*, int,
                                     hipStream_t);

}  // namespace octohydro
