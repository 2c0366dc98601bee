// Forward kernels for (uint8_t input, int accumulator).
#include "fht_launch.h"

namespace fht {
hipError_t launch_pass_u8(const PassLaunch& L, hipStream_t s) { return launch_pass_t<uint8_t, int>(L, s); }
hipError_t launch_engine_u8(const EngineArgs& A, int G, int grid, hipStream_t s)
{
    return launch_engine_t<uint8_t, int>(A, G, grid, s);
}
hipError_t launch_direct_u8(const PassLaunch& L, int k, hipStream_t s) { return launch_direct_t<uint8_t, int>(L, k, s); }
hipError_t launch_table_u8(const EngineGroup* table, int n_groups, int n_items, const int* group_of, int G,
                          bool first, bool last,
                          int rows, hipStream_t s)
{
    return launch_table_t<uint8_t, int>(table, n_groups, n_items, group_of, G, first, last, rows, s);
}
hipError_t launch_table_direct_u8(const EngineGroup* table, int n_groups, int n_items, hipStream_t s)
{
    return launch_table_direct_t<uint8_t, int>(table, n_groups, n_items, s);
}
}  // namespace fht
