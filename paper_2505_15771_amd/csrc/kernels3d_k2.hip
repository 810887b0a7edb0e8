// Three-dimensional stage, trace and energy kernels of degree k = 2 (templates in stage3d.h).
#include "stage3d.h"

namespace hho {
template hipError_t launch_stage3<2, double>(const StageArgs<double> &, int, hipStream_t);
template hipError_t launch_traces3<2, double>(const StageArgs<double> &, int, hipStream_t);
template hipError_t launch_energy3<2, double>(const StageArgs<double> &, int, hipStream_t);
template hipError_t launch_stage3<2, float>(const StageArgs<float> &, int, hipStream_t);
template hipError_t launch_traces3<2, float>(const StageArgs<float> &, int, hipStream_t);
template hipError_t launch_energy3<2, float>(const StageArgs<float> &, int, hipStream_t);
}  // namespace hho
