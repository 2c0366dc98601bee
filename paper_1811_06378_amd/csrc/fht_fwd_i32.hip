// Forward kernels for (int input, int accumulator).
#include "fht_launch.h"

namespace fht {
hipError_t launch_pass_i32(const PassLaunch& L, hipStream_t s) { return launch_pass_t<int, int>(L, s); }
hipError_t launch_engine_i32(const EngineArgs& A, int G, int grid, hipStream_t s)
{
    return launch_engine_t<int, int>(A, G, grid, s);
}
hipError_t launch_direct_i32(const PassLaunch& L, int k, hipStream_t s) { return launch_direct_t<int, int>(L, k, s); }
hipError_t launch_table_i32(const EngineGroup* table, int n_groups, int n_items, const int* group_of, int G,
                          bool first, bool last,
                          int rows, hipStream_t s)
{
    return launch_table_t<int, int>(table, n_groups, n_items, group_of, G, first, last, rows, s);
}
hipError_t launch_table_direct_i32(const EngineGroup* table, int n_groups, int n_items, hipStream_t s)
{
    return launch_table_direct_t<int, int>(table, n_groups, n_items, s);
}
}  // namespace fht
