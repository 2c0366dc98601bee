// Type dispatch of the pass launchers, plus the fhtshift and fill kernels'
// launchers.
#include "fht_launch.h"

#include <cstdlib>

namespace fht {

__global__ void fht_zero_kernel(uint32_t* p, int64_t rows, int64_t cols_words, int64_t ld_words)
{
    const int64_t total = rows * cols_words;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / cols_words, c = i - r * cols_words;
        p[r * ld_words + c] = 0u;
    }
}

// dtype codes: 0 = u8, 1 = i32, 2 = f32
static hipError_t launch_pass_typed(const PassLaunch& L, int in_t, int acc_t, int op, hipStream_t s)
{
    if (op == 1) {
        if (in_t == 0 && acc_t == 1) return launch_pass_max_u8(L, s);
        if (in_t == 1 && acc_t == 1) return launch_pass_max_i32(L, s);
        if (in_t == 2 && acc_t == 2) return launch_pass_max_f32(L, s);
        return hipErrorInvalidValue;
    }
    if (op != 0) return hipErrorInvalidValue;
    if (in_t == 0 && acc_t == 1) return launch_pass_u8(L, s);
    if (in_t == 1 && acc_t == 1) return launch_pass_i32(L, s);
    if (in_t == 2 && acc_t == 2) return launch_pass_f32(L, s);
    return hipErrorInvalidValue;
}

hipError_t launch_pass(const PassLaunch& L, int in_t, int acc_t, hipStream_t s, int op)
{
    int slot = -1;
    if (timing_on()) {
        // template arguments as the kernel has them: ..., op, waves per tile,
        // first-pass source mode (0 plain, 1 sheared rows, 2 element loads)
        const PassDesc& d = L.d[0];
        const bool first = d.src_kind != SRC_BAND;
        const int mode = !first ? 0 : d.scale_num != 0 ? 2 : d.S1 == 0 ? 0 : d.src_kind == SRC_IMAGE ? 1 : 2;
        std::string name = kernel_name("fht_pass_kernel", in_t, acc_t, d.G - 3, first, d.dst_kind == DST_HOUGH, op,
                                       d.tile_rows / 8);
        name.insert(name.size() - 1, ", " + std::to_string(mode));
        slot = timing_begin(name, s);
    }
    const hipError_t e = launch_pass_typed(L, in_t, acc_t, op, s);
    timing_end(slot, s);
    return e;
}

hipError_t launch_engine(const EngineArgs& A, int G, int grid, int in_t, int acc_t, hipStream_t s)
{
    if (in_t == 0 && acc_t == 1) return launch_engine_u8(A, G, grid, s);
    if (in_t == 1 && acc_t == 1) return launch_engine_i32(A, G, grid, s);
    if (in_t == 2 && acc_t == 2) return launch_engine_f32(A, G, grid, s);
    return hipErrorInvalidValue;
}

static hipError_t launch_table_typed(const EngineGroup* table, int n_groups, int n_items, const int* group_of,
                                     int G, bool first, bool last, int rows, int in_t, int acc_t, hipStream_t s)
{
    if (in_t == 0 && acc_t == 1) return launch_table_u8(table, n_groups, n_items, group_of, G, first, last, rows, s);
    if (in_t == 1 && acc_t == 1) return launch_table_i32(table, n_groups, n_items, group_of, G, first, last, rows, s);
    if (in_t == 2 && acc_t == 2) return launch_table_f32(table, n_groups, n_items, group_of, G, first, last, rows, s);
    return hipErrorInvalidValue;
}

hipError_t launch_table(const EngineGroup* table, int n_groups, int n_items, const int* group_of, int G, bool first,
                        bool last, int rows, int in_t, int acc_t, hipStream_t s)
{
    int slot = -1;
    if (timing_on())
        slot = timing_begin(kernel_name("fht_table_kernel", in_t, acc_t, G - 3, first, last, -1, rows / 8), s);
    const hipError_t e = launch_table_typed(table, n_groups, n_items, group_of, G, first, last, rows, in_t, acc_t, s);
    timing_end(slot, s);
    return e;
}

hipError_t launch_table_direct(const EngineGroup* table, int n_groups, int n_items, int in_t, int acc_t,
                               hipStream_t s)
{
    if (in_t == 0 && acc_t == 1) return launch_table_direct_u8(table, n_groups, n_items, s);
    if (in_t == 1 && acc_t == 1) return launch_table_direct_i32(table, n_groups, n_items, s);
    if (in_t == 2 && acc_t == 2) return launch_table_direct_f32(table, n_groups, n_items, s);
    return hipErrorInvalidValue;
}

hipError_t launch_direct(const PassLaunch& L, int k, int in_t, int acc_t, hipStream_t s, int op)
{
    if (op == 1) {
        if (in_t == 0 && acc_t == 1) return launch_direct_max_u8(L, k, s);
        if (in_t == 1 && acc_t == 1) return launch_direct_max_i32(L, k, s);
        if (in_t == 2 && acc_t == 2) return launch_direct_max_f32(L, k, s);
        return hipErrorInvalidValue;
    }
    if (op != 0) return hipErrorInvalidValue;
    if (in_t == 0 && acc_t == 1) return launch_direct_u8(L, k, s);
    if (in_t == 1 && acc_t == 1) return launch_direct_i32(L, k, s);
    if (in_t == 2 && acc_t == 2) return launch_direct_f32(L, k, s);
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint_pass(const AdjLaunch& L, int t, hipStream_t s)
{
    int slot = -1;
    if (timing_on()) {
        // the kernel's template arguments: type, GB, first, last, accumulate
        std::string name = kernel_name("fht_adj_pass_kernel", -1, t, L.d[0].G - 3, L.d[0].src_kind == 0,
                                       L.d[0].dst_kind != 0);
        name.insert(name.size() - 1, (L.d[0].dst_kind != 0 && L.d[0].accumulate) ? ", true" : ", false");
        slot = timing_begin(name, s);
    }
    hipError_t e = hipErrorInvalidValue;
    if (t == 1) e = launch_adj_pass_i32(L, s);
    if (t == 2) e = launch_adj_pass_f32(L, s);
    timing_end(slot, s);
    return e;
}

hipError_t launch_adjoint_pair(const AdjLaunch& L, int t, hipStream_t s)
{
    int slot = -1;
    if (timing_on()) {
        // the kernel's template arguments: type, GB, first, accumulate
        std::string name = kernel_name("fht_adj_pair_kernel", -1, t, L.d[0].G - 3, L.d[0].src_kind == 0,
                                       L.d[0].accumulate != 0);
        slot = timing_begin(name, s);
    }
    hipError_t e = hipErrorInvalidValue;
    if (t == 1) e = launch_adj_pair_i32(L, s);
    if (t == 2) e = launch_adj_pair_f32(L, s);
    timing_end(slot, s);
    return e;
}

hipError_t launch_adjoint_direct(const AdjLaunch& L, int k, int t, hipStream_t s)
{
    if (t == 1) return launch_adj_direct_i32(L, k, s);
    if (t == 2) return launch_adj_direct_f32(L, k, s);
    return hipErrorInvalidValue;
}

// Persistent grid: two 512-thread workgroups per CU (LDS and registers both
// allow two), on the current device.
int engine_grid_size()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 512;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 512;
    return 2 * cus;
}

hipError_t launch_zero(void* p, int64_t rows, int64_t cols, int64_t ld, int elem_bytes, hipStream_t s)
{
    if (elem_bytes != 4) return hipErrorInvalidValue;
    const int64_t total = rows * cols;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fht_zero_kernel, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, rows, cols, ld);
    return hipGetLastError();
}

hipError_t launch_unshear(const void* a0, int W, int n, int S1, void* img, int64_t ld_img, int w, int h,
                          int transposed, int elem_bytes, hipStream_t s)
{
    if (elem_bytes != 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fht_unshear_kernel<uint32_t>, dim3((w + 255) / 256, h < 65535 ? h : 65535), dim3(256), 0, s,
                       (const uint32_t*)a0, W, n, S1, (uint32_t*)img, ld_img, w, h, transposed);
    return hipGetLastError();
}

hipError_t launch_shift(const void* in, int64_t ld_in, void* out, int64_t ld_out, int elem_bytes,
                        int hp, int wp, int inverse, hipStream_t s)
{
    if (elem_bytes != 4) return hipErrorInvalidValue;
    const int W = hp + wp;
    const int rows = 2 * (hp + wp) - 3;
    if (in == out && ld_in == ld_out) {
        const size_t lds_bytes = (size_t)W * 4;
        static bool attr_set = false;
        if (!attr_set) {
            hipError_t e = hipFuncSetAttribute((const void*)fht_shift_inplace_kernel<uint32_t>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
            if (e != hipSuccess) return e;
            attr_set = true;
        }
        hipLaunchKernelGGL(fht_shift_inplace_kernel<uint32_t>, dim3(rows), dim3(1024), lds_bytes, s,
                           (uint32_t*)out, ld_out, hp, wp, inverse);
    } else {
        hipLaunchKernelGGL(fht_shift_kernel<uint32_t>, dim3((W + 1023) / 1024, rows < 65535 ? rows : 65535), dim3(256), 0, s,
                           (const uint32_t*)in, ld_in, (uint32_t*)out, ld_out, hp, wp, inverse);
    }
    return hipGetLastError();
}

}  // namespace fht
