// Forward pass kernels for (int input, int accumulator).
#include "fht_launch.h"

namespace fht {
hipError_t launch_pass_i32(const PassLaunch& L, int G, bool first, bool last, hipStream_t s)
{
    return launch_pass_t<int, int>(L, G, first, last, s);
}
hipError_t launch_direct_i32(const PassLaunch& L, int k, hipStream_t s) { return launch_direct_t<int, int>(L, k, s); }
}  // namespace fht
