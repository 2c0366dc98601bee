// Forward kernels for (float input, float accumulator).
#include "fht_launch.h"

namespace fht {
hipError_t launch_pass_f32(const PassLaunch& L, hipStream_t s) { return launch_pass_t<float, float>(L, s); }
hipError_t launch_engine_f32(const EngineArgs& A, int G, int grid, hipStream_t s)
{
    return launch_engine_t<float, float>(A, G, grid, s);
}
hipError_t launch_direct_f32(const PassLaunch& L, int k, hipStream_t s) { return launch_direct_t<float, float>(L, k, s); }
hipError_t launch_table_f32(const EngineGroup* table, int n_groups, int n_items, const int* group_of, int G,
                          bool first, bool last,
                          int rows, hipStream_t s)
{
    return launch_table_t<float, float>(table, n_groups, n_items, group_of, G, first, last, rows, s);
}
hipError_t launch_table_direct_f32(const EngineGroup* table, int n_groups, int n_items, hipStream_t s)
{
    return launch_table_direct_t<float, float>(table, n_groups, n_items, s);
}
}  // namespace fht
