// Adjoint kernels for the int accumulator.
#include "fht_launch.h"

namespace fht {
hipError_t launch_adj_pass_i32(const AdjLaunch& L, hipStream_t s) { return launch_adj_pass_t<int>(L, s); }
hipError_t launch_adj_pair_i32(const AdjLaunch& L, hipStream_t s) { return launch_adj_pair_t<int>(L, s); }
hipError_t launch_adj_direct_i32(const AdjLaunch& L, int k, hipStream_t s) { return launch_adj_direct_t<int>(L, k, s); }
}  // namespace fht
