// Forward kernels of the max transform for (float input, float accumulator).
#include "fht_launch.h"

namespace fht {
hipError_t launch_pass_max_f32(const PassLaunch& L, hipStream_t s) { return launch_pass_t<float, float, 1>(L, s); }
hipError_t launch_direct_max_f32(const PassLaunch& L, int k, hipStream_t s)
{
    return launch_direct_t<float, float, 1>(L, k, s);
}
}  // namespace fht
