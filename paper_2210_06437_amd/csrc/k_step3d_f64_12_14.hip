// Instantiations of the 3D step kernel k_step3d, binary64, 12 to 14
// fields: one of the units its instantiations are spread over so that they
// compile in parallel.
#include "octohydro_kernels3d.h"

namespace octohydro {

template hipError_t launch_step3d_one<double, 12>(const StepArgs&, int, const double*, int,
                                     hipStream_t);
template hipError_t launch_step3d_one<double, 13>(const StepArgs&, int, const double*, int,
                                     hipStream_t);
template hipError_t launch_step3d_one<double, 14>(const StepArgs&, int, const double*, int,
                                     hipStream_t);

}  // namespace octohydro
