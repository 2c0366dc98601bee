// Forward kernels of the max transform for (unsigned char input, int accumulator).
#include "fht_launch.h"

namespace fht {
hipError_t launch_pass_max_u8(const PassLaunch& L, hipStream_t s) { return launch_pass_t<unsigned char, int, 1>(L, s); }
hipError_t launch_direct_max_u8(const PassLaunch& L, int k, hipStream_t s)
{
    return launch_direct_t<unsigned char, int, 1>(L, k, s);
}
}  // namespace fht
