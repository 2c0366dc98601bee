// Device code of the dyadic Fast Hough Transform for gfx950 (CDNA4): the
// kernel templates, instantiated per element type in fht_inst_*.hip.
//
// The transform of one quadrant is the stage recurrence of Brady's FHT
// (arXiv 1811.06378, section 2 and section 4 / Fig. 6): after stage j the rows
// form blocks of 2^(j+1); stage j merges two neighbouring blocks,
//   A[j+1][b*2^(j+1) + t][x] = A[j][b*2^(j+1) + (t>>1)][x]
//                            + A[j][b*2^(j+1) + 2^j + (t>>1)][x + dir*(t - (t>>1))]   (mod W).
//
// Stage fusion.  G consecutive stages starting at stage j0 regroup exactly:
// with u < 2^j0, m, v < 2^G,
//   A[j0+G][B*2^(j0+G) + u*2^G + v][x]
//     = MiniFHT_G( m -> A[j0][B*2^(j0+G) + m*2^j0 + u][x + dir*u*m] )[v][x],
// i.e. the same G-stage transform on the 2^G rows m*2^j0 + u, each read with a
// per-row column offset dir*u*m.  Applied twice inside a tile (G = 3 + GB):
// the first 3 stages run on 8 contiguous rows held by one wave, the last GB
// stages on rows 8g + u' read back from LDS with offsets dir*u'*g.
//
// Register layout.  A workgroup (8 waves) holds 64 rows x 512 columns; a lane
// owns 8 consecutive columns of 8 rows.  A stage's column shift (at most 4 in
// registers) reads the lane's own registers or, across the lane boundary, the
// neighbouring lane's registers through a DPP wavefront shift by one lane, so
// the shift costs no LDS traffic.  The rightmost (leftmost for dir = -1)
// 2^G - 1 columns of a tile are halo: computed, not stored.
//
// No MFMA: the recurrence is a bandwidth-bound chain of additions.

#pragma once

#include "fht_internal.h"

#include <climits>

namespace fht {

// ------------------------------------------------------------ small helpers

__device__ __forceinline__ int wrap_once(int e, int W)
{
    // e in [0, W + 512): one conditional subtraction covers W >= 512
    if (e >= W) e -= W;
    if (e >= W) e %= W;
    return e;
}

__device__ __forceinline__ int mod_pos(long long a, int W)
{
    long long r = a % W;
    return (int)(r < 0 ? r + W : r);
}

// floor((2*y*S1 + (n-1)) / (2*(n-1))): the horizontal shear of row y for an
// inclination range (section 4), rounded half up.
__device__ __forceinline__ int shear_of_row(int y, int S1, int n)
{
    if (S1 == 0 || n <= 1) return 0;
    long long num = 2LL * y * S1 + (n - 1);
    long long den = 2LL * (n - 1);
    long long q = num / den;
    if ((num % den != 0) && (num < 0)) q -= 1;
    return (int)q;
}

// Lane i reads lane i+1 (DPP wave_shl:1) / lane i-1 (DPP wave_shr:1).
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
constexpr int kDppFromNext = 0x130;  // wave_shl:1
constexpr int kDppFromPrev = 0x138;  // wave_shr:1

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, dpp_move<CTRL>(__builtin_bit_cast(int, v)));
}

template <typename T> __device__ __forceinline__ T to_acc(uint8_t v) { return (T)v; }
template <typename T> __device__ __forceinline__ T to_acc(int v) { return (T)v; }
template <typename T> __device__ __forceinline__ T to_acc(float v) { return (T)v; }

// --------------------------------------------------------- register stages

// Forward stage J on 8 register rows: blocks of 2^(J+1) rows, block rows
// t = 0..2^(J+1)-1 from rows (t>>1) and 2^J + (t>>1), the latter shifted by
// dir*(t - (t>>1)) columns.
template <typename T, int DIR, int J>
__device__ __forceinline__ void fwd_stage(T (&a)[8][8])
{
    constexpr int H = 1 << J;
    T o[8][8];
#pragma unroll
    for (int blk = 0; blk < 8; blk += 2 * H) {
#pragma unroll
        for (int t = 0; t < 2 * H; ++t) {
            const int sub = t >> 1;
            const int d = t - sub;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int cc = c + DIR * d;
                T bot;
                if (cc >= 8) bot = dpp_move<kDppFromNext>(a[blk + H + sub][cc - 8]);
                else if (cc < 0) bot = dpp_move<kDppFromPrev>(a[blk + H + sub][cc + 8]);
                else bot = a[blk + H + sub][cc];
                o[blk + t][c] = a[blk + sub][c] + bot;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) a[r][c] = o[r][c];
}

// Transpose of fwd_stage: input row t of a merged block goes back to the two
// rows it was summed from, so
//   top[i][x]    = g[2i][x] + g[2i+1][x]
//   bottom[u][x] = g[2u][x - dir*u] + g[2u+1][x - dir*(u+1)].
template <typename T, int DIR, int J>
__device__ __forceinline__ void adj_stage(T (&a)[8][8])
{
    constexpr int H = 1 << J;
    T o[8][8];
#pragma unroll
    for (int blk = 0; blk < 8; blk += 2 * H) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
#pragma unroll
            for (int c = 0; c < 8; ++c) o[blk + i][c] = a[blk + 2 * i][c] + a[blk + 2 * i + 1][c];
        }
#pragma unroll
        for (int u = 0; u < H; ++u) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                T x0, x1;
                {
                    const int cc = c - DIR * u;
                    if (cc >= 8) x0 = dpp_move<kDppFromNext>(a[blk + 2 * u][cc - 8]);
                    else if (cc < 0) x0 = dpp_move<kDppFromPrev>(a[blk + 2 * u][cc + 8]);
                    else x0 = a[blk + 2 * u][cc];
                }
                {
                    const int cc = c - DIR * (u + 1);
                    if (cc >= 8) x1 = dpp_move<kDppFromNext>(a[blk + 2 * u + 1][cc - 8]);
                    else if (cc < 0) x1 = dpp_move<kDppFromPrev>(a[blk + 2 * u + 1][cc + 8]);
                    else x1 = a[blk + 2 * u + 1][cc];
                }
                o[blk + H + u][c] = x0 + x1;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) a[r][c] = o[r][c];
}

template <typename T, int DIR, int GB>
__device__ __forceinline__ void fwd_stages_b(T (&b)[8][8])
{
    if constexpr (GB > 0) fwd_stage<T, DIR, 0>(b);
    if constexpr (GB > 1) fwd_stage<T, DIR, 1>(b);
    if constexpr (GB > 2) fwd_stage<T, DIR, 2>(b);
}

template <typename T, int DIR, int GB>
__device__ __forceinline__ void adj_stages_b(T (&b)[8][8])
{
    if constexpr (GB > 2) adj_stage<T, DIR, 2>(b);
    if constexpr (GB > 1) adj_stage<T, DIR, 1>(b);
    if constexpr (GB > 0) adj_stage<T, DIR, 0>(b);
}

__device__ __forceinline__ int lds_index(int tile_row, int col)
{
    // column-swizzled: column col of a row lives in plane (col & 7) at (col >> 3),
    // so both the lane-contiguous stores and the offset loads hit 64 distinct banks
    return tile_row * kLdsRow + (col & 7) * kPlane + (col >> 3);
}

// ------------------------------------------------------------ source loads

// Padded source value at quadrant row R, for the 8 columns owned by this lane
// starting at logical column x (any integer; taken mod W).
template <typename TIn, typename T>
__device__ __forceinline__ void load_row(const PassDesc& d, int R, long long x, T (&v)[8])
{
    const int W = d.W;
    if (d.src_kind == SRC_BAND) {
        const T* band = reinterpret_cast<const T*>(d.src) + (long long)R * d.src_ld;
        int e0 = mod_pos(x + d.src_off, W);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            int e = wrap_once(e0 + c, W);
            v[c] = (e < d.src_bw) ? band[e] : (T)0;
        }
        return;
    }
    const TIn* img = reinterpret_cast<const TIn*>(d.src);
    const int sh = shear_of_row(R, d.S1, d.n);
    int e0 = mod_pos(x - sh, W);
    if (d.src_kind == SRC_IMAGE) {
        const bool row_ok = R < d.img_h;
        const TIn* p = img + (long long)R * d.src_ld;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            int e = wrap_once(e0 + c, W);
            v[c] = (row_ok && e < d.img_w) ? to_acc<T>(p[e]) : (T)0;
        }
    } else {  // SRC_IMAGE_T: quadrant row R is image column R
        const bool col_ok = R < d.img_w;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            int e = wrap_once(e0 + c, W);
            v[c] = (col_ok && e < d.img_h) ? to_acc<T>(img[(long long)e * d.src_ld + R]) : (T)0;
        }
    }
}

// ------------------------------------------------------ fused forward pass

template <typename TIn, typename T, int GB, int DIR>
__device__ __forceinline__ void fwd_tile(const PassDesc& d, int rt, int win, T* lds)
{
    constexpr int G = 3 + GB;
    constexpr int NMINI = 1 << (6 - G);          // mini-transforms of 2^G rows per tile
    constexpr int VW = kWinCols - (1 << G);      // stored columns per tile
    constexpr int LOFF = DIR > 0 ? 0 : kLdsOffNeg;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int j0 = d.j0;
    const int n_mini = d.n >> G;
    const long long x_lo = (long long)d.x_start + (long long)win * VW;
    const long long xw0 = x_lo - (DIR < 0 ? (1 << G) : 0);

    // ---- phase A: 8 contiguous mini rows per wave, first 3 stages
    T a[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int tr = wave * 8 + r;
        const int t = tr >> G;
        const int m = tr & ((1 << G) - 1);
        const int mu = rt * NMINI + t;
        const int B = mu >> j0;
        const int u = mu & ((1 << j0) - 1);
        const bool active = (mu < n_mini) && ((u << G) <= d.row_limit);
        if (active) {
            const int R = (B << (j0 + G)) + (m << j0) + u;
            load_row<TIn, T>(d, R, xw0 + 8 * lane + (long long)DIR * u * m, a[r]);
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) a[r][c] = (T)0;
        }
    }
    fwd_stage<T, DIR, 0>(a);
    fwd_stage<T, DIR, 1>(a);
    fwd_stage<T, DIR, 2>(a);
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) lds[lds_index(wave * 8 + r, 8 * lane + c + LOFF)] = a[r][c];
    __syncthreads();

    // ---- phase B: rows 8g + u' with offsets dir*u'*g, last GB stages
    T b[8][8];
#pragma unroll
    for (int rho = 0; rho < 8; ++rho) {
        const int rp = rho & ((1 << GB) - 1);
        const int q = rho >> GB;
        const int kappa = (wave << (3 - GB)) + q;
        const int t = kappa >> 3;
        const int up = kappa & 7;
        const int tr = (t << G) + (rp << 3) + up;
        const int off = DIR * up * rp + LOFF;
#pragma unroll
        for (int c = 0; c < 8; ++c) b[rho][c] = lds[lds_index(tr, 8 * lane + c + off)];
    }
    fwd_stages_b<T, DIR, GB>(b);

    // ---- store
    const int wc0 = 8 * lane;
    const bool lane_ok = DIR > 0 ? (wc0 < VW) : (wc0 >= (1 << G));
    if (!lane_ok) return;
    const long long x0 = xw0 + wc0;
#pragma unroll
    for (int rho = 0; rho < 8; ++rho) {
        const int rp = rho & ((1 << GB) - 1);
        const int q = rho >> GB;
        const int kappa = (wave << (3 - GB)) + q;
        const int t = kappa >> 3;
        const int up = kappa & 7;
        const int mu = rt * NMINI + t;
        if (mu >= n_mini) continue;
        const int B = mu >> j0;
        const int u = mu & ((1 << j0) - 1);
        const int s_local = (u << G) + (up << GB) + rp;
        if (s_local > d.row_limit) continue;
        const int out_row = (B << (j0 + G)) + s_local;
        if (d.dst_kind == DST_BAND) {
            T* dst = reinterpret_cast<T*>(d.dst) + (long long)out_row * d.dst_ld;
            const long long e0 = x0 + d.dst_off;
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (e0 + c < d.dst_bw) dst[e0 + c] = b[rho][c];
        } else {
            const int s = out_row;
            if (s == d.skip_row) continue;
            T* dst = reinterpret_cast<T*>(d.dst) + (long long)(d.row_base + d.row_sign * s) * d.dst_ld;
            const int roll = d.shifted ? ((d.roll_a + d.roll_b * s) >> 1) : 0;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const long long x = x0 + c;
                if (x < d.W) dst[wrap_once((int)x + roll, d.W)] = b[rho][c];
            }
        }
    }
}

template <typename TIn, typename T, int GB>
__global__ __launch_bounds__(kThreads) void fht_pass_kernel(const PassLaunch L)
{
    __shared__ T lds[kTileRows * kLdsRow];
    const PassDesc& d = L.d[blockIdx.z];
    if ((int)blockIdx.x >= d.n_windows || (int)blockIdx.y >= d.n_row_tiles) return;
    if (d.dir > 0) fwd_tile<TIn, T, GB, 1>(d, blockIdx.y, blockIdx.x, lds);
    else fwd_tile<TIn, T, GB, -1>(d, blockIdx.y, blockIdx.x, lds);
}

// -------------------------------------------- direct form for n <= 4 rows

template <typename TIn, typename T>
__device__ __forceinline__ T src_value(const PassDesc& d, int R, int x)
{
    const int W = d.W;
    const int e = mod_pos((long long)x - shear_of_row(R, d.S1, d.n), W);
    const TIn* img = reinterpret_cast<const TIn*>(d.src);
    if (d.src_kind == SRC_IMAGE)
        return (R < d.img_h && e < d.img_w) ? to_acc<T>(img[(long long)R * d.src_ld + e]) : (T)0;
    return (R < d.img_w && e < d.img_h) ? to_acc<T>(img[(long long)e * d.src_ld + R]) : (T)0;
}

// The same add tree as K stages of the recurrence, evaluated top-down.
template <typename TIn, typename T, int K>
__device__ T direct_sum(const PassDesc& d, int base, int s, int x)
{
    if constexpr (K == 0) {
        return src_value<TIn, T>(d, base, x);
    } else {
        const int sub = s >> 1;
        const T top = direct_sum<TIn, T, K - 1>(d, base, sub, x);
        const T bot = direct_sum<TIn, T, K - 1>(d, base + (1 << (K - 1)), sub,
                                               mod_pos((long long)x + d.dir * (s - sub), d.W));
        return top + bot;
    }
}

template <typename TIn, typename T, int K>
__global__ __launch_bounds__(256) void fht_direct_kernel(const PassLaunch L)
{
    const PassDesc& d = L.d[blockIdx.z];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (x >= d.W || s >= d.n || s > d.row_limit || s == d.skip_row) return;
    const T v = direct_sum<TIn, T, K>(d, 0, s, x);
    T* dst = reinterpret_cast<T*>(d.dst) + (long long)(d.row_base + d.row_sign * s) * d.dst_ld;
    const int roll = d.shifted ? ((d.roll_a + d.roll_b * s) >> 1) : 0;
    dst[mod_pos((long long)x + roll, d.W)] = v;
}

// ------------------------------------------------------ fused adjoint pass
//
// The transpose of one forward pass: the 2^G rows u*2^G + v of a block are
// read contiguously, the mini transform runs backwards (last GB stages
// transposed, then the LDS exchange with offsets moved to the write side, then
// the first 3 stages transposed) and row m is written with its column offset
// dir*u*m added.

template <typename T>
__device__ __forceinline__ void adj_load_row(const AdjDesc& d, int s_row, long long x, T (&v)[8])
{
    const int W = d.W;
    if (d.src_kind == 1) {  // band
        const T* band = reinterpret_cast<const T*>(d.src) + (long long)s_row * d.src_ld;
        int e0 = mod_pos(x + d.src_off, W);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            int e = wrap_once(e0 + c, W);
            v[c] = (e < d.src_bw) ? band[e] : (T)0;
        }
        return;
    }
    // Hough gradient: quadrant row s -> Hough row, shifted columns
    if (s_row == d.skip_row) {
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = (T)0;
        return;
    }
    const T* src = reinterpret_cast<const T*>(d.src) + (long long)(d.row_base + d.row_sign * s_row) * d.src_ld;
    const int roll = d.shifted ? ((d.roll_a + d.roll_b * s_row) >> 1) : 0;
    int e0 = mod_pos(x + roll, W);
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = src[wrap_once(e0 + c, W)];
}

template <typename T, int GB, int DIR>
__device__ __forceinline__ void adj_tile(const AdjDesc& d, int rt, int win, T* lds)
{
    constexpr int G = 3 + GB;
    constexpr int NMINI = 1 << (6 - G);
    constexpr int VW = kWinCols - (1 << G);
    // transposed shifts point the other way, so the halo sits on the other side
    constexpr int LOFF = DIR > 0 ? 0 : kLdsOffNeg;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int j0 = d.j0;
    const int n_mini = d.n >> G;
    const long long x_lo = (long long)d.x_start + (long long)win * VW;
    const long long xw0 = x_lo - (DIR > 0 ? (1 << G) : 0);

    // ---- load the forward pass's output rows (contiguous within a block)
    T b[8][8];
#pragma unroll
    for (int rho = 0; rho < 8; ++rho) {
        const int rp = rho & ((1 << GB) - 1);
        const int q = rho >> GB;
        const int kappa = (wave << (3 - GB)) + q;
        const int t = kappa >> 3;
        const int up = kappa & 7;
        const int mu = rt * NMINI + t;
        if (mu < n_mini) {
            const int B = mu >> j0;
            const int u = mu & ((1 << j0) - 1);
            const int s_row = (B << (j0 + G)) + (u << G) + (up << GB) + rp;
            adj_load_row<T>(d, s_row, xw0 + 8 * lane, b[rho]);
        } else {
#pragma unroll
            for (int c = 0; c < 8; ++c) b[rho][c] = (T)0;
        }
    }
    adj_stages_b<T, DIR, GB>(b);
#pragma unroll
    for (int rho = 0; rho < 8; ++rho) {
        const int rp = rho & ((1 << GB) - 1);
        const int q = rho >> GB;
        const int kappa = (wave << (3 - GB)) + q;
        const int t = kappa >> 3;
        const int up = kappa & 7;
        const int tr = (t << G) + (rp << 3) + up;
        const int off = DIR * up * rp + LOFF;
#pragma unroll
        for (int c = 0; c < 8; ++c) lds[lds_index(tr, 8 * lane + c + off)] = b[rho][c];
    }
    __syncthreads();

    T a[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) a[r][c] = lds[lds_index(wave * 8 + r, 8 * lane + c + LOFF)];
    adj_stage<T, DIR, 2>(a);
    adj_stage<T, DIR, 1>(a);
    adj_stage<T, DIR, 0>(a);

    // ---- store row m of each mini transform at its offset dir*u*m
    const int wc0 = 8 * lane;
    const bool lane_ok = DIR > 0 ? (wc0 >= (1 << G)) : (wc0 < VW);
    if (!lane_ok) return;
    const long long x0 = xw0 + wc0;  // logical column of register 0 before the offset
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int tr = wave * 8 + r;
        const int t = tr >> G;
        const int m = tr & ((1 << G) - 1);
        const int mu = rt * NMINI + t;
        if (mu >= n_mini) continue;
        const int B = mu >> j0;
        const int u = mu & ((1 << j0) - 1);
        const int R = (B << (j0 + G)) + (m << j0) + u;
        const long long xo = x0 + (long long)DIR * u * m;
        if (d.dst_kind == 0) {
            // band: window columns are band positions x_lo..; the offset moves them
            T* dst = reinterpret_cast<T*>(d.dst) + (long long)R * d.dst_ld;
            // the windows cover window columns [0, W) once; column z of row m
            // lands on z + dir*u*m, a bijection of the cyclic row
            const int e0 = mod_pos(xo + d.dst_off, d.W);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (x0 + c < (long long)d.W) {
                    const int e = wrap_once(e0 + c, d.W);
                    if (e < d.dst_bw) dst[e] = a[r][c];
                }
            }
        } else {
            // image: the first forward pass has u = 0, so no offset remains
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const long long x = x0 + c;
                if (d.dst_kind == 1) {
                    if (R < d.img_h && x >= 0 && x < d.img_w) {
                        T* p = reinterpret_cast<T*>(d.dst) + (long long)R * d.dst_ld + x;
                        *p = d.accumulate ? (T)(*p + a[r][c]) : a[r][c];
                    }
                } else {
                    if (R < d.img_w && x >= 0 && x < d.img_h) {
                        T* p = reinterpret_cast<T*>(d.dst) + (long long)x * d.dst_ld + R;
                        *p = d.accumulate ? (T)(*p + a[r][c]) : a[r][c];
                    }
                }
            }
        }
    }
}

template <typename T, int GB>
__global__ __launch_bounds__(kThreads) void fht_adj_pass_kernel(const AdjLaunch L)
{
    __shared__ T lds[kTileRows * kLdsRow];
    const AdjDesc& d = L.d[blockIdx.z];
    if ((int)blockIdx.x >= d.n_windows || (int)blockIdx.y >= d.n_row_tiles) return;
    if (d.dir > 0) adj_tile<T, GB, 1>(d, blockIdx.y, blockIdx.x, lds);
    else adj_tile<T, GB, -1>(d, blockIdx.y, blockIdx.x, lds);
}

// Adjoint for n <= 4 rows: B_j from B_{j+1} by the transposed stage, top-down.
template <typename T, int J, int K>
__device__ T adj_direct(const AdjDesc& d, int row, int x)
{
    if constexpr (J == K) {
        T v[8];
        adj_load_row<T>(d, row, x, v);  // only v[0] is used
        return v[0];
    } else {
        const int blk = 1 << J;
        const int base = (row / (2 * blk)) * (2 * blk);
        const int i = row - base;
        if (i < blk) {
            return adj_direct<T, J + 1, K>(d, base + 2 * i, x) + adj_direct<T, J + 1, K>(d, base + 2 * i + 1, x);
        }
        const int u = i - blk;
        return adj_direct<T, J + 1, K>(d, base + 2 * u, mod_pos((long long)x - d.dir * u, d.W)) +
               adj_direct<T, J + 1, K>(d, base + 2 * u + 1, mod_pos((long long)x - d.dir * (u + 1), d.W));
    }
}

template <typename T, int K>
__global__ __launch_bounds__(256) void fht_adj_direct_kernel(const AdjLaunch L)
{
    const AdjDesc& d = L.d[blockIdx.z];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int R = blockIdx.y;
    if (R >= d.n) return;
    const int cols = d.dst_kind == 1 ? d.img_w : d.img_h;
    const int rows = d.dst_kind == 1 ? d.img_h : d.img_w;
    if (x >= cols || R >= rows) return;
    const T v = adj_direct<T, 0, K>(d, R, x);
    T* p = d.dst_kind == 1 ? reinterpret_cast<T*>(d.dst) + (long long)R * d.dst_ld + x
                           : reinterpret_cast<T*>(d.dst) + (long long)x * d.dst_ld + R;
    *p = d.accumulate ? (T)(*p + v) : v;
}

// ------------------------------------------------------------- fhtshift

// Roll of full-image row r (section 5): quadrant and local shift from the row
// index, then floor((n +- s)/2).
__device__ __forceinline__ int row_roll(int r, int hp, int wp)
{
    if (r < hp) return (hp + (hp - 1 - r)) >> 1;                 // q1, s = h'-1-r
    if (r < 2 * hp - 1) return (hp - (r - hp + 1)) >> 1;         // q2, s = r-h'+1
    if (r < 2 * hp + wp - 2) return (wp - (2 * hp + wp - 3 - r)) >> 1;  // q3
    return (wp + (r - (2 * hp + wp - 3))) >> 1;                  // q4
}

template <typename T>
__global__ __launch_bounds__(1024) void fht_shift_inplace_kernel(T* buf, int64_t ld, int hp, int wp, int inverse)
{
    extern __shared__ unsigned char smem_raw[];
    T* row = reinterpret_cast<T*>(smem_raw);
    const int W = hp + wp;
    const int r = blockIdx.x;
    T* p = buf + (long long)r * ld;
    for (int x = threadIdx.x; x < W; x += blockDim.x) row[x] = p[x];
    __syncthreads();
    int roll = row_roll(r, hp, wp) % W;
    if (inverse) roll = (W - roll) % W;
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
        int src = x - roll;
        if (src < 0) src += W;
        p[x] = row[src];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void fht_shift_kernel(const T* in, int64_t ld_in, T* out, int64_t ld_out,
                                                        int hp, int wp, int inverse)
{
    const int W = hp + wp;
    const int r = blockIdx.y;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W) return;
    int roll = row_roll(r, hp, wp) % W;
    if (inverse) roll = (W - roll) % W;
    int src = x - roll;
    if (src < 0) src += W;
    out[(long long)r * ld_out + x] = in[(long long)r * ld_in + src];
}

}  // namespace fht
