// Forward pass kernels for (uint8_t input, int accumulator).
#include "fht_launch.h"

namespace fht {
hipError_t launch_pass_u8(const PassLaunch& L, int G, bool first, bool last, hipStream_t s)
{
    return launch_pass_t<uint8_t, int>(L, G, first, last, s);
}
hipError_t launch_direct_u8(const PassLaunch& L, int k, hipStream_t s) { return launch_direct_t<uint8_t, int>(L, k, s); }
}  // namespace fht
