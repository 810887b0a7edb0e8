// Three-dimensional stage, trace and energy kernels of degree k = 1 (templates in stage3d.h).
#include "stage3d.h"

namespace hho {
template hipError_t launch_stage3<1, double>(const StageArgs<double> &, int, hipStream_t);
template hipError_t launch_traces3<1, double>(const StageArgs<double> &, int, hipStream_t);
template hipError_t launch_energy3<1, double>(const StageArgs<double> &, int, hipStream_t);
template hipError_t launch_stage3<1, float>(const StageArgs<float> &, int, hipStream_t);
template hipError_t launch_traces3<1, float>(const StageArgs<float> &, int, hipStream_t);
template hipError_t launch_energy3<1, float>(const StageArgs<float> &, int, hipStream_t);
}  // namespace hho
