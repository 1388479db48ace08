// Instantiations of the 3D step kernel k_step3d, binary32 storage, 9 to 11
// fields: one of the units its instantiations are spread over so that they
// compile in parallel.
#include "octohydro_kernels3d.h"

namespace octohydro {

template hipError_t launch_step3d_one<float, 9>(const StepArgs&, int, const float*, int,
                                     hipStream_t);
template hipError_t launch_step3d_one<float, 10>(const StepArgs&, int, const float*, int,
                                     hipStream_t);
template hipError_t launch_step3d_one<float, 11>(const StepArgs&, int, const float*, int,
                                     hipStream_t);

}  // namespace octohydro
