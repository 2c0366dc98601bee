// Launch templates of the pass kernels; each element type is instantiated in
// its own translation unit (fht_fwd_*.hip, fht_adj_*.hip) so they compile in
// parallel.
#pragma once

#include "fht_device.h"

namespace fht {

inline dim3 pass_grid(const PassLaunch& L)
{
    int wx = 1, ry = 1;
    for (int i = 0; i < L.nd; ++i) {
        wx = L.d[i].n_windows > wx ? L.d[i].n_windows : wx;
        ry = L.d[i].n_row_tiles > ry ? L.d[i].n_row_tiles : ry;
    }
    return dim3(wx, ry, L.nd);
}

template <typename TIn, typename T, bool FIRST, bool LAST>
hipError_t launch_pass_fl(const PassLaunch& L, int G, hipStream_t s)
{
    const dim3 grid = pass_grid(L);
    switch (G) {
    case 3: hipLaunchKernelGGL((fht_pass_kernel<TIn, T, 0, FIRST, LAST>), grid, dim3(kThreads), 0, s, L); break;
    case 4: hipLaunchKernelGGL((fht_pass_kernel<TIn, T, 1, FIRST, LAST>), grid, dim3(kThreads), 0, s, L); break;
    case 5: hipLaunchKernelGGL((fht_pass_kernel<TIn, T, 2, FIRST, LAST>), grid, dim3(kThreads), 0, s, L); break;
    case 6: hipLaunchKernelGGL((fht_pass_kernel<TIn, T, 3, FIRST, LAST>), grid, dim3(kThreads), 0, s, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// first = the pass reads the image, last = the pass writes the Hough image
template <typename TIn, typename T>
hipError_t launch_pass_t(const PassLaunch& L, int G, bool first, bool last, hipStream_t s)
{
    if (first) return last ? launch_pass_fl<TIn, T, true, true>(L, G, s) : launch_pass_fl<TIn, T, true, false>(L, G, s);
    if constexpr (sizeof(TIn) == sizeof(T)) {
        return last ? launch_pass_fl<T, T, false, true>(L, G, s) : launch_pass_fl<T, T, false, false>(L, G, s);
    }
    return hipErrorInvalidValue;
}

template <typename TIn, typename T>
hipError_t launch_direct_t(const PassLaunch& L, int k, hipStream_t s)
{
    int W = 1, n = 1;
    for (int i = 0; i < L.nd; ++i) {
        W = L.d[i].W > W ? L.d[i].W : W;
        n = L.d[i].n > n ? L.d[i].n : n;
    }
    const dim3 grid((W + 255) / 256, n, L.nd);
    switch (k) {
    case 0: hipLaunchKernelGGL((fht_direct_kernel<TIn, T, 0>), grid, dim3(256), 0, s, L); break;
    case 1: hipLaunchKernelGGL((fht_direct_kernel<TIn, T, 1>), grid, dim3(256), 0, s, L); break;
    case 2: hipLaunchKernelGGL((fht_direct_kernel<TIn, T, 2>), grid, dim3(256), 0, s, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, bool FIRST, bool LAST>
hipError_t launch_adj_pass_fl(const AdjLaunch& L, int G, hipStream_t s)
{
    int wx = 1, ry = 1;
    for (int i = 0; i < L.nd; ++i) {
        wx = L.d[i].n_windows > wx ? L.d[i].n_windows : wx;
        ry = L.d[i].n_row_tiles > ry ? L.d[i].n_row_tiles : ry;
    }
    const dim3 grid(wx, ry, L.nd);
    switch (G) {
    case 3: hipLaunchKernelGGL((fht_adj_pass_kernel<T, 0, FIRST, LAST>), grid, dim3(kThreads), 0, s, L); break;
    case 4: hipLaunchKernelGGL((fht_adj_pass_kernel<T, 1, FIRST, LAST>), grid, dim3(kThreads), 0, s, L); break;
    case 5: hipLaunchKernelGGL((fht_adj_pass_kernel<T, 2, FIRST, LAST>), grid, dim3(kThreads), 0, s, L); break;
    case 6: hipLaunchKernelGGL((fht_adj_pass_kernel<T, 3, FIRST, LAST>), grid, dim3(kThreads), 0, s, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// first = reads the Hough gradient, last = writes the image gradient
template <typename T>
hipError_t launch_adj_pass_t(const AdjLaunch& L, int G, bool first, bool last, hipStream_t s)
{
    if (first) return last ? launch_adj_pass_fl<T, true, true>(L, G, s) : launch_adj_pass_fl<T, true, false>(L, G, s);
    return last ? launch_adj_pass_fl<T, false, true>(L, G, s) : launch_adj_pass_fl<T, false, false>(L, G, s);
}

template <typename T>
hipError_t launch_adj_direct_t(const AdjLaunch& L, int k, hipStream_t s)
{
    int cols = 1, n = 1;
    for (int i = 0; i < L.nd; ++i) {
        const int c = L.d[i].dst_kind == 1 ? L.d[i].img_w : L.d[i].img_h;
        cols = c > cols ? c : cols;
        n = L.d[i].n > n ? L.d[i].n : n;
    }
    const dim3 grid((cols + 255) / 256, n, L.nd);
    switch (k) {
    case 0: hipLaunchKernelGGL((fht_adj_direct_kernel<T, 0>), grid, dim3(256), 0, s, L); break;
    case 1: hipLaunchKernelGGL((fht_adj_direct_kernel<T, 1>), grid, dim3(256), 0, s, L); break;
    case 2: hipLaunchKernelGGL((fht_adj_direct_kernel<T, 2>), grid, dim3(256), 0, s, L); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// per-type entry points (defined in the instantiation units)
hipError_t launch_pass_u8(const PassLaunch& L, int G, bool first, bool last, hipStream_t s);
hipError_t launch_pass_i32(const PassLaunch& L, int G, bool first, bool last, hipStream_t s);
hipError_t launch_pass_f32(const PassLaunch& L, int G, bool first, bool last, hipStream_t s);
hipError_t launch_direct_u8(const PassLaunch& L, int k, hipStream_t s);
hipError_t launch_direct_i32(const PassLaunch& L, int k, hipStream_t s);
hipError_t launch_direct_f32(const PassLaunch& L, int k, hipStream_t s);
hipError_t launch_adj_pass_i32(const AdjLaunch& L, int G, bool first, bool last, hipStream_t s);
hipError_t launch_adj_pass_f32(const AdjLaunch& L, int G, bool first, bool last, hipStream_t s);
hipError_t launch_adj_direct_i32(const AdjLaunch& L, int k, hipStream_t s);
hipError_t launch_adj_direct_f32(const AdjLaunch& L, int k, hipStream_t s);

}  // namespace fht
