// Forward pass kernels for (float input, float accumulator).
#include "fht_launch.h"

namespace fht {
hipError_t launch_pass_f32(const PassLaunch& L, int G, bool first, bool last, hipStream_t s)
{
    return launch_pass_t<float, float>(L, G, first, last, s);
}
hipError_t launch_direct_f32(const PassLaunch& L, int k, hipStream_t s) { return launch_direct_t<float, float>(L, k, s); }
}  // namespace fht
