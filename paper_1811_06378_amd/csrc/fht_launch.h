// Launch templates of the kernels; each element type is instantiated in its
// own translation unit (fht_fwd_*.hip, fht_adj_*.hip) so they compile in
// parallel.
#pragma once

#include "fht_device.h"

namespace fht {

template <typename TIn, typename T, int GB, int OP, int NW>
hipError_t launch_pass_g(const PassLaunch& L0, hipStream_t s)
{
    PassLaunch L = L0;
    L.n_tiles = 0;
    for (int i = 0; i < L.nd; ++i) L.n_tiles += L.d[i].n_row_tiles * L.d[i].n_windows;
    if (L.n_tiles == 0) return hipSuccess;
    const bool first = L.d[0].src_kind != SRC_BAND, last = L.d[0].dst_kind == DST_HOUGH;
    const dim3 grid((L.n_tiles + kXcds - 1) / kXcds * kXcds, L.n_img > 0 ? L.n_img : 1), block(NW * 64);
    // first passes of sheared or scaled sources (angle range, sum only) take
    // the kernel with their source path; every descriptor of a launch agrees
    int mode = 0;
    for (int i = 0; i < L.nd; ++i) {
        const PassDesc& d = L.d[i];
        const int m = !first ? 0 : d.scale_num != 0 ? 2 : d.S1 == 0 ? 0 : d.src_kind == SRC_IMAGE ? 1 : 2;
        if (i > 0 && m != mode) return hipErrorInvalidValue;
        mode = m;
    }
    if (mode != 0) {
        if constexpr (OP == 0) {
            if (mode == 1 && last)
                hipLaunchKernelGGL((fht_pass_kernel<TIn, T, GB, true, true, OP, NW, 1>), grid, block, 0, s, L);
            else if (mode == 1)
                hipLaunchKernelGGL((fht_pass_kernel<TIn, T, GB, true, false, OP, NW, 1>), grid, block, 0, s, L);
            else if (last)
                hipLaunchKernelGGL((fht_pass_kernel<TIn, T, GB, true, true, OP, NW, 2>), grid, block, 0, s, L);
            else
                hipLaunchKernelGGL((fht_pass_kernel<TIn, T, GB, true, false, OP, NW, 2>), grid, block, 0, s, L);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (first && last)
        hipLaunchKernelGGL((fht_pass_kernel<TIn, T, GB, true, true, OP, NW, 0>), grid, block, 0, s, L);
    else if (first)
        hipLaunchKernelGGL((fht_pass_kernel<TIn, T, GB, true, false, OP, NW, 0>), grid, block, 0, s, L);
    else if (last)
        hipLaunchKernelGGL((fht_pass_kernel<TIn, T, GB, false, true, OP, NW, 0>), grid, block, 0, s, L);
    else
        hipLaunchKernelGGL((fht_pass_kernel<TIn, T, GB, false, false, OP, NW, 0>), grid, block, 0, s, L);
    return hipGetLastError();
}

// all descriptors of one launch share G, first/last and the tile height;
// 32-row tiles exist for passes of at most 5 stages
template <typename TIn, typename T, int OP = 0>
hipError_t launch_pass_t(const PassLaunch& L, hipStream_t s)
{
    const bool narrow = L.d[0].tile_rows == kNarrowRows;
    switch (L.d[0].G) {
    case 3: return narrow ? launch_pass_g<TIn, T, 0, OP, 4>(L, s) : launch_pass_g<TIn, T, 0, OP, 8>(L, s);
    case 4: return narrow ? launch_pass_g<TIn, T, 1, OP, 4>(L, s) : launch_pass_g<TIn, T, 1, OP, 8>(L, s);
    case 5: return narrow ? launch_pass_g<TIn, T, 2, OP, 4>(L, s) : launch_pass_g<TIn, T, 2, OP, 8>(L, s);
    case 6: return narrow ? hipErrorInvalidValue : launch_pass_g<TIn, T, 3, OP, 8>(L, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename TIn, typename T, int GB>
hipError_t launch_engine_g(const EngineArgs& A, int grid, hipStream_t s)
{
    if (A.table) hipLaunchKernelGGL((fht_engine_kernel<TIn, T, GB, false>), dim3(grid), dim3(kThreads), 0, s, A);
    else hipLaunchKernelGGL((fht_engine_kernel<TIn, T, GB, true>), dim3(grid), dim3(kThreads), 0, s, A);
    return hipGetLastError();
}

template <typename TIn, typename T, int GB, int NW>
hipError_t launch_table_g(const EngineGroup* table, int n_groups, int n_items, const int* group_of, bool first,
                          bool last, hipStream_t s)
{
    const dim3 grid((n_items + kXcds - 1) / kXcds * kXcds), block(NW * 64);
    if (first && last)
        hipLaunchKernelGGL((fht_table_kernel<TIn, T, GB, true, true, NW>), grid, block, 0, s, table, n_groups, n_items,
                           group_of);
    else if (first)
        hipLaunchKernelGGL((fht_table_kernel<TIn, T, GB, true, false, NW>), grid, block, 0, s, table, n_groups, n_items,
                           group_of);
    else if (last)
        hipLaunchKernelGGL((fht_table_kernel<TIn, T, GB, false, true, NW>), grid, block, 0, s, table, n_groups, n_items,
                           group_of);
    else
        hipLaunchKernelGGL((fht_table_kernel<TIn, T, GB, false, false, NW>), grid, block, 0, s, table, n_groups,
                           n_items, group_of);
    return hipGetLastError();
}

template <typename TIn, typename T>
hipError_t launch_table_t(const EngineGroup* table, int n_groups, int n_items, const int* group_of, int G, bool first,
                          bool last, int rows, hipStream_t s)
{
    const bool narrow = rows == kNarrowRows;
    switch (G) {
    case 3:
        return narrow ? launch_table_g<TIn, T, 0, 4>(table, n_groups, n_items, group_of, first, last, s)
                      : launch_table_g<TIn, T, 0, 8>(table, n_groups, n_items, group_of, first, last, s);
    case 4:
        return narrow ? launch_table_g<TIn, T, 1, 4>(table, n_groups, n_items, group_of, first, last, s)
                      : launch_table_g<TIn, T, 1, 8>(table, n_groups, n_items, group_of, first, last, s);
    case 5:
        return narrow ? launch_table_g<TIn, T, 2, 4>(table, n_groups, n_items, group_of, first, last, s)
                      : launch_table_g<TIn, T, 2, 8>(table, n_groups, n_items, group_of, first, last, s);
    case 6: return narrow ? hipErrorInvalidValue : launch_table_g<TIn, T, 3, 8>(table, n_groups, n_items, group_of, first, last, s);
    default: return hipErrorInvalidValue;
    }
}

// every group of one engine launch has G = 3 + GB
template <typename TIn, typename T>
hipError_t launch_engine_t(const EngineArgs& A, int G, int grid, hipStream_t s)
{
    switch (G) {
    case 3: return launch_engine_g<TIn, T, 0>(A, grid, s);
    case 4: return launch_engine_g<TIn, T, 1>(A, grid, s);
    case 5: return launch_engine_g<TIn, T, 2>(A, grid, s);
    case 6: return launch_engine_g<TIn, T, 3>(A, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename TIn, typename T>
hipError_t launch_table_direct_t(const EngineGroup* table, int n_groups, int n_items, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL((fht_table_direct_kernel<TIn, T>), dim3((n_items + 255) / 256), dim3(256), 0, s, table,
                       n_groups, n_items);
    return hipGetLastError();
}

template <typename TIn, typename T, int OP = 0>
hipError_t launch_direct_t(const PassLaunch& L, int k, hipStream_t s)
{
    int W = 1, n = 1;
    for (int i = 0; i < L.nd; ++i) {
        W = L.d[i].W > W ? L.d[i].W : W;
        n = L.d[i].n > n ? L.d[i].n : n;
    }
    const dim3 grid((W + 255) / 256, n, L.nd * (L.n_img > 0 ? L.n_img : 1));
    switch (k) {
    case 0: hipLaunchKernelGGL((fht_direct_kernel<TIn, T, 0, OP>), grid, dim3(256), 0, s, L); break;
    case 1: hipLaunchKernelGGL((fht_direct_kernel<TIn, T, 1, OP>), grid, dim3(256), 0, s, L); break;
    case 2: hipLaunchKernelGGL((fht_direct_kernel<TIn, T, 2, OP>), grid, dim3(256), 0, s, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int GB>
hipError_t launch_adj_pass_g(const AdjLaunch& L, hipStream_t s)
{
    int wx = 1, ry = 1;
    for (int i = 0; i < L.nd; ++i) {
        wx = L.d[i].n_windows > wx ? L.d[i].n_windows : wx;
        ry = L.d[i].n_row_tiles > ry ? L.d[i].n_row_tiles : ry;
    }
    const bool first = L.d[0].src_kind == 0, last = L.d[0].dst_kind != 0;
    const dim3 grid(wx, ry, L.nd * (L.n_img > 0 ? L.n_img : 1));
    // image passes that add to the stored gradient run their own instantiation; all
    // descriptors of a launch agree
    const bool acc = last && L.d[0].accumulate != 0;
    for (int i = 1; i < L.nd; ++i)
        if ((last && L.d[i].accumulate != 0) != acc) return hipErrorInvalidValue;
    if (first && last && acc)
        hipLaunchKernelGGL((fht_adj_pass_kernel<T, GB, true, true, true>), grid, dim3(kThreads), 0, s, L);
    else if (first && last)
        hipLaunchKernelGGL((fht_adj_pass_kernel<T, GB, true, true, false>), grid, dim3(kThreads), 0, s, L);
    else if (first)
        hipLaunchKernelGGL((fht_adj_pass_kernel<T, GB, true, false, false>), grid, dim3(kThreads), 0, s, L);
    else if (last && acc)
        hipLaunchKernelGGL((fht_adj_pass_kernel<T, GB, false, true, true>), grid, dim3(kThreads), 0, s, L);
    else if (last)
        hipLaunchKernelGGL((fht_adj_pass_kernel<T, GB, false, true, false>), grid, dim3(kThreads), 0, s, L);
    else
        hipLaunchKernelGGL((fht_adj_pass_kernel<T, GB, false, false, false>), grid, dim3(kThreads), 0, s, L);
    return hipGetLastError();
}

// all descriptors of one launch share G and first/last
template <typename T>
hipError_t launch_adj_pass_t(const AdjLaunch& L, hipStream_t s)
{
    switch (L.d[0].G) {
    case 3: return launch_adj_pass_g<T, 0>(L, s);
    case 4: return launch_adj_pass_g<T, 1>(L, s);
    case 5: return launch_adj_pass_g<T, 2>(L, s);
    case 6: return launch_adj_pass_g<T, 3>(L, s);
    default: return hipErrorInvalidValue;
    }
}

// Mirror-pair image passes: descriptors (U, M) at 2z and 2z + 1, U
// unmirrored and M mirrored, of one quadrant geometry each (same n, stage
// split, row tiles, windows and image target); all pairs share G, the
// first-pass flag and the accumulate flag.
template <typename T, int GB>
hipError_t launch_adj_pair_g(const AdjLaunch& L, hipStream_t s)
{
    if (L.nd < 2 || (L.nd & 1)) return hipErrorInvalidValue;
    int wx = 1, ry = 1;
    for (int i = 0; i < L.nd; i += 2) {
        const AdjDesc& u = L.d[i];
        const AdjDesc& m = L.d[i + 1];
        if (u.mirror != 0 || m.mirror != 1 || u.n != m.n || u.G != m.G || u.j0 != 0 || m.j0 != 0 ||
            u.n_windows != m.n_windows || u.n_row_tiles != m.n_row_tiles || u.dst_kind == 0 ||
            u.dst_kind != m.dst_kind || u.dst != m.dst || u.W != m.W || u.x_start != 0 ||
            u.src_kind != L.d[0].src_kind || m.src_kind != L.d[0].src_kind ||
            u.accumulate != L.d[0].accumulate || u.G != L.d[0].G)
            return hipErrorInvalidValue;
        wx = u.n_windows > wx ? u.n_windows : wx;
        ry = u.n_row_tiles > ry ? u.n_row_tiles : ry;
    }
    const bool first = L.d[0].src_kind == 0, acc = L.d[0].accumulate != 0;
    const dim3 grid(wx, ry, (L.nd / 2) * (L.n_img > 0 ? L.n_img : 1)), block(2 * kThreads);
    if (first && acc) hipLaunchKernelGGL((fht_adj_pair_kernel<T, GB, true, true>), grid, block, 0, s, L);
    else if (first) hipLaunchKernelGGL((fht_adj_pair_kernel<T, GB, true, false>), grid, block, 0, s, L);
    else if (acc) hipLaunchKernelGGL((fht_adj_pair_kernel<T, GB, false, true>), grid, block, 0, s, L);
    else hipLaunchKernelGGL((fht_adj_pair_kernel<T, GB, false, false>), grid, block, 0, s, L);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_pair_t(const AdjLaunch& L, hipStream_t s)
{
    switch (L.d[0].G) {
    case 3: return launch_adj_pair_g<T, 0>(L, s);
    case 4: return launch_adj_pair_g<T, 1>(L, s);
    case 5: return launch_adj_pair_g<T, 2>(L, s);
    case 6: return launch_adj_pair_g<T, 3>(L, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_adj_direct_t(const AdjLaunch& L, int k, hipStream_t s)
{
    int cols = 1, n = 1;
    for (int i = 0; i < L.nd; ++i) {
        const int c = L.d[i].dst_kind == 1 ? L.d[i].img_w : (L.d[i].dst_kind == 2 ? L.d[i].img_h : L.d[i].W);
        cols = c > cols ? c : cols;
        n = L.d[i].n > n ? L.d[i].n : n;
    }
    const dim3 grid((cols + 255) / 256, n, L.nd * (L.n_img > 0 ? L.n_img : 1));
    switch (k) {
    case 0: hipLaunchKernelGGL((fht_adj_direct_kernel<T, 0>), grid, dim3(256), 0, s, L); break;
    case 1: hipLaunchKernelGGL((fht_adj_direct_kernel<T, 1>), grid, dim3(256), 0, s, L); break;
    case 2: hipLaunchKernelGGL((fht_adj_direct_kernel<T, 2>), grid, dim3(256), 0, s, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// per-type entry points (defined in the instantiation units)
#define FHT_DECLARE_FWD(name)                                                   \
    hipError_t launch_pass_##name(const PassLaunch& L, hipStream_t s);           \
    hipError_t launch_pass_max_##name(const PassLaunch& L, hipStream_t s);       \
    hipError_t launch_direct_max_##name(const PassLaunch& L, int k, hipStream_t s); \
    hipError_t launch_engine_##name(const EngineArgs& A, int G, int grid, hipStream_t s); \
    hipError_t launch_direct_##name(const PassLaunch& L, int k, hipStream_t s);                 \
    hipError_t launch_table_##name(const EngineGroup* table, int n_groups, int n_items, const int* group_of, int G, \
                                   bool first, bool last, int rows, hipStream_t s);                      \
    hipError_t launch_table_direct_##name(const EngineGroup* table, int n_groups, int n_items, hipStream_t s);
FHT_DECLARE_FWD(u8)
FHT_DECLARE_FWD(i32)
FHT_DECLARE_FWD(f32)
#undef FHT_DECLARE_FWD
hipError_t launch_adj_pass_i32(const AdjLaunch& L, hipStream_t s);
hipError_t launch_adj_pass_f32(const AdjLaunch& L, hipStream_t s);
hipError_t launch_adj_pair_i32(const AdjLaunch& L, hipStream_t s);
hipError_t launch_adj_pair_f32(const AdjLaunch& L, hipStream_t s);
hipError_t launch_adj_direct_i32(const AdjLaunch& L, int k, hipStream_t s);
hipError_t launch_adj_direct_f32(const AdjLaunch& L, int k, hipStream_t s);

}  // namespace fht
