// Instantiations of the 3D step kernel k_step3d, binary64, 9 to 11
// fields: one of the units its instantiations are spread over so that they
// compile in parallel.
#include "octohydro_kernels3d.h"

namespace octohydro {

template hipError_t launch_step3d_one<double, 9>(const StepArgs&, int, const double*, int,
                                     hipStream_t);
template hipError_t launch_step3d_one<double, 10>(const StepArgs&, int, const double*, int,
                                     hipStream_t);
template hipError_t launch_step3d_one<double, 11>(const StepArgs&, int, const double*, int,
                                     hipStream_t);

}  // namespace octohydro
