// Adjoint kernels for the float accumulator.
#include "fht_launch.h"

namespace fht {
hipError_t launch_adj_pass_f32(const AdjLaunch& L, hipStream_t s) { return launch_adj_pass_t<float>(L, s); }
hipError_t launch_adj_pair_f32(const AdjLaunch& L, hipStream_t s) { return launch_adj_pair_t<float>(L, s); }
hipError_t launch_adj_direct_f32(const AdjLaunch& L, int k, hipStream_t s) { return launch_adj_direct_t<float>(L, k, s); }
}  // namespace fht
