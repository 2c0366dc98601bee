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
// Forward stage J on 8 register rows: blocks of 2^(J+1) rows; block rows
// 2i and 2i+1 both come from the pair (top row i, bottom row 2^J + i), the
// bottom one shifted by dir*i and dir*(i+1) columns.  Each output pair
// depends on one input pair only, so the stage is a set of row butterflies.
template <typename T, int DIR, int J>
__device__ __forceinline__ void fwd_stage(T (&a)[8][8])
{
    constexpr int H = 1 << J;
    T o[8][8];
#pragma unroll
    for (int blk = 0; blk < 8; blk += 2 * H) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const T (&top)[8] = a[blk + i];
            const T (&bot)[8] = a[blk + H + i];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                int c0 = c + DIR * i, c1 = c + DIR * (i + 1);
                T b0, b1;
                if (c0 >= 8) b0 = dpp_move<kDppFromNext>(bot[c0 - 8]);
                else if (c0 < 0) b0 = dpp_move<kDppFromPrev>(bot[c0 + 8]);
                else b0 = bot[c0];
                if (c1 >= 8) b1 = dpp_move<kDppFromNext>(bot[c1 - 8]);
                else if (c1 < 0) b1 = dpp_move<kDppFromPrev>(bot[c1 + 8]);
                else b1 = bot[c1];
                o[blk + 2 * i][c] = top[c] + b0;
                o[blk + 2 * i + 1][c] = top[c] + b1;
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

// LDS rows are column-swizzled: column x lives in plane (x & 7) at slot
// (x >> 3), so lane-contiguous 8-column groups and offset reads both spread
// over all banks.  A row segment starting at a wave-uniform offset is
// accessed through one base address plus compile-time immediates: the
// residue (off & 7) selects one of 8 unrolled patterns.
template <int O7, typename T>
__device__ __forceinline__ void lds_read8_fixed(const T* p, T (&v)[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = p[((c + O7) & 7) * kPlane + ((c + O7) >> 3)];
}

template <int O7, typename T>
__device__ __forceinline__ void lds_write8_fixed(T* p, const T (&v)[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c) p[((c + O7) & 7) * kPlane + ((c + O7) >> 3)] = v[c];
}

// row_lane = row base + lane; off >= 0 (wave-uniform)
template <typename T>
__device__ __forceinline__ void lds_read8(const T* row_lane, int off, T (&v)[8])
{
    const T* p = row_lane + (off >> 3);
    switch (off & 7) {
    case 0: lds_read8_fixed<0>(p, v); break;
    case 1: lds_read8_fixed<1>(p, v); break;
    case 2: lds_read8_fixed<2>(p, v); break;
    case 3: lds_read8_fixed<3>(p, v); break;
    case 4: lds_read8_fixed<4>(p, v); break;
    case 5: lds_read8_fixed<5>(p, v); break;
    case 6: lds_read8_fixed<6>(p, v); break;
    default: lds_read8_fixed<7>(p, v); break;
    }
}

template <typename T>
__device__ __forceinline__ void lds_write8(T* row_lane, int off, const T (&v)[8])
{
    T* p = row_lane + (off >> 3);
    switch (off & 7) {
    case 0: lds_write8_fixed<0>(p, v); break;
    case 1: lds_write8_fixed<1>(p, v); break;
    case 2: lds_write8_fixed<2>(p, v); break;
    case 3: lds_write8_fixed<3>(p, v); break;
    case 4: lds_write8_fixed<4>(p, v); break;
    case 5: lds_write8_fixed<5>(p, v); break;
    case 6: lds_write8_fixed<6>(p, v); break;
    default: lds_write8_fixed<7>(p, v); break;
    }
}

__device__ __forceinline__ int lds_index(int tile_row, int col)
{
    // column-swizzled: column col of a row lives in plane (col & 7) at (col >> 3),
    // so both the lane-contiguous stores and the offset loads hit 64 distinct banks
    return tile_row * kLdsRow + (col & 7) * kPlane + (col >> 3);
}

// ------------------------------------------------------------ vector access

typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
typedef int i32x4u __attribute__((ext_vector_type(4), aligned(4)));
typedef unsigned int u32x2u __attribute__((ext_vector_type(2), aligned(4)));

template <typename T> struct vec4u;
template <> struct vec4u<float> { typedef f32x4u type; };
template <> struct vec4u<int> { typedef i32x4u type; };

// 8 consecutive elements.  Only dword alignment is required: gfx950 serves
// dword-aligned 16-byte vector accesses, which the pre-rolled rows need.
template <typename T>
__device__ __forceinline__ void load8(const T* p, T (&v)[8])
{
    typedef typename vec4u<T>::type V;
    const V a = *reinterpret_cast<const V*>(p);
    const V b = *reinterpret_cast<const V*>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

template <typename T>
__device__ __forceinline__ void store8(T* p, const T (&v)[8])
{
    typedef typename vec4u<T>::type V;
    V a, b;
    a.x = v[0]; a.y = v[1]; a.z = v[2]; a.w = v[3];
    b.x = v[4]; b.y = v[5]; b.z = v[6]; b.w = v[7];
    *reinterpret_cast<V*>(p) = a;
    *reinterpret_cast<V*>(p + 4) = b;
}

// Streaming store for the final Hough image (written once, never re-read here).
template <typename T>
__device__ __forceinline__ void store8_stream(T* p, const T (&v)[8])
{
    typedef typename vec4u<T>::type V;
    V a, b;
    a.x = v[0]; a.y = v[1]; a.z = v[2]; a.w = v[3];
    b.x = v[4]; b.y = v[5]; b.z = v[6]; b.w = v[7];
    __builtin_nontemporal_store(a, reinterpret_cast<V*>(p));
    __builtin_nontemporal_store(b, reinterpret_cast<V*>(p + 4));
}

template <typename TIn>
__device__ __forceinline__ bool vec_ok(const TIn* p)
{
    if constexpr (sizeof(TIn) == 1) return (reinterpret_cast<uintptr_t>(p) & 3) == 0;
    else return true;
}

template <typename TIn, typename T>
__device__ __forceinline__ void load8_src(const TIn* p, T (&v)[8])
{
    if constexpr (sizeof(TIn) == 1) {
        const u32x2u w = *reinterpret_cast<const u32x2u*>(p);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v[c] = (T)((w.x >> (8 * c)) & 0xFFu);
            v[4 + c] = (T)((w.y >> (8 * c)) & 0xFFu);
        }
    } else {
        load8<T>(reinterpret_cast<const T*>(p), v);
    }
}

template <typename T>
__device__ __forceinline__ void zero8(T (&v)[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = (T)0;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// a mod W for a wave-uniform a (the pass geometry keeps |a| < 4W whenever
// W >= 1024; small W takes the division).
__device__ __forceinline__ int mod_w(int a, int W)
{
    if (W >= 1024 && a > -4 * W && a < 4 * W) {
        a += 4 * W;
        if (a >= 4 * W) a -= 4 * W;
        if (a >= 2 * W) a -= 2 * W;
        if (a >= W) a -= W;
        return a;
    }
    int r = a % W;
    return r < 0 ? r + W : r;
}

// e in [0, W + 512) -> e mod W
__device__ __forceinline__ int wrap_lane(int e, int W)
{
    if (e >= W) e -= W;
    if (e >= W) e %= W;
    return e;
}

// ------------------------------------------------------------ source loads
//
// Loads are issued for all rows before any result is used: lanes whose 8
// columns lie inside the data read them with two 16-byte loads, lanes whose 8
// columns are all zero padding read a static zero page, and only lanes that
// straddle a boundary (rare) are patched element by element afterwards.  An
// if/else per row would make every row wait for the previous row's loads.

static __device__ __attribute__((aligned(64))) unsigned int g_zero_page[16];

template <typename T>
__device__ __forceinline__ const T* zero_page()
{
    return reinterpret_cast<const T*>(g_zero_page);
}

// Band row R: returns the lane's first band index and whether it needs a patch.
template <typename T>
__device__ __forceinline__ bool issue_band_row(const PassDesc& d, int R, int xrow, int lane, T (&v)[8], int& e0)
{
    const int W = d.W;
    const T* band = reinterpret_cast<const T*>(d.src) + (long long)R * d.src_ld;
    e0 = wrap_lane(mod_w(xrow + d.src_off, W) + 8 * lane, W);
    const bool fast = e0 + 8 <= d.src_bw;
    const bool zero = e0 >= d.src_bw && e0 + 8 <= W;
    load8<T>(fast ? band + e0 : zero_page<T>(), v);
    return !fast && !zero;
}

template <typename T>
__device__ __forceinline__ void patch_band_row(const PassDesc& d, int R, int e0, T (&v)[8])
{
    const int W = d.W;
    const T* band = reinterpret_cast<const T*>(d.src) + (long long)R * d.src_ld;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        int e = e0 + c;
        if (e >= W) e -= W;
        v[c] = (e < d.src_bw) ? band[e] : (T)0;
    }
}

// Image row R (quadrants 1, 2; sheared for the angle range).
template <typename TIn, typename T>
__device__ __forceinline__ bool issue_image_row(const PassDesc& d, int R, int xrow, int lane, T (&v)[8], int& e0)
{
    const int W = d.W;
    const TIn* p = reinterpret_cast<const TIn*>(d.src) + (long long)R * d.src_ld;
    e0 = wrap_lane(mod_w(xrow - shear_of_row(R, d.S1, d.n), W) + 8 * lane, W);
    const bool row_ok = R < d.img_h;
    const bool fast = row_ok && e0 + 8 <= d.img_w && vec_ok<TIn>(p + e0);
    const bool zero = !row_ok || (e0 >= d.img_w && e0 + 8 <= W);
    load8_src<TIn, T>(fast ? p + e0 : zero_page<TIn>(), v);
    return !fast && !zero;
}

template <typename TIn, typename T>
__device__ __forceinline__ void patch_image_row(const PassDesc& d, int R, int e0, T (&v)[8])
{
    const int W = d.W;
    const TIn* img = reinterpret_cast<const TIn*>(d.src);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        int e = e0 + c;
        if (e >= W) e -= W;
        if (d.src_kind == SRC_IMAGE)
            v[c] = (R < d.img_h && e < d.img_w) ? to_acc<T>(img[(long long)R * d.src_ld + e]) : (T)0;
        else
            v[c] = (R < d.img_w && e < d.img_h) ? to_acc<T>(img[(long long)e * d.src_ld + R]) : (T)0;
    }
}

// Transposed image (quadrants 3, 4) with a shear: element loads only.
template <typename TIn, typename T>
__device__ __forceinline__ bool issue_image_t_row(const PassDesc& d, int R, int xrow, int lane, T (&v)[8], int& e0)
{
    e0 = wrap_lane(mod_w(xrow - shear_of_row(R, d.S1, d.n), d.W) + 8 * lane, d.W);
    zero8(v);
    return true;
}

// Rows R0..R0+7 of the transposed image (image columns), unsheared: for each
// of the lane's 8 columns (image rows) the 8 values are contiguous in memory.
template <typename TIn, typename T>
__device__ __forceinline__ void load_rows_transposed(const PassDesc& d, int R0, int xrow, int lane, T (&a)[8][8])
{
    const int W = d.W;
    const int e0 = wrap_lane(mod_w(xrow, W) + 8 * lane, W);
    const TIn* img = reinterpret_cast<const TIn*>(d.src);
    const bool all_cols = R0 + 8 <= d.img_w;
    T t[8][8];
    bool patch[8];
    bool any = false;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        int e = e0 + c;
        if (e >= W) e -= W;
        const TIn* p = img + (long long)e * d.src_ld + R0;
        const bool inside = e < d.img_h;
        const bool fast = inside && all_cols && vec_ok<TIn>(p);
        load8_src<TIn, T>(fast ? p : zero_page<TIn>(), t[c]);
        patch[c] = inside && !fast;
        any |= patch[c];
    }
    if (__any(any)) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (patch[c]) {
                int e = e0 + c;
                if (e >= W) e -= W;
                const TIn* p = img + (long long)e * d.src_ld + R0;
#pragma unroll
                for (int r = 0; r < 8; ++r) t[c][r] = (R0 + r < d.img_w) ? to_acc<T>(p[r]) : (T)0;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int r = 0; r < 8; ++r) a[r][c] = t[c][r];
}

// ------------------------------------------------------ fused forward pass

template <typename TIn, typename T, int GB, int DIR, bool FIRST, bool LAST>
__device__ __forceinline__ void fwd_tile(const PassDesc& d, int rt, int win, T* lds)
{
    constexpr int G = 3 + GB;
    constexpr int NMINI = 1 << (6 - G);          // mini-transforms of 2^G rows per tile
    constexpr int VW = kWinCols - (1 << G);      // stored columns per tile
    constexpr int LOFF = DIR > 0 ? 0 : kLdsOffNeg;
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    const int j0 = d.j0;
    const int n_mini = d.n >> G;
    const int x_lo = d.x_start + win * VW;
    const int xw0 = x_lo - (DIR < 0 ? (1 << G) : 0);

    // ---- phase A: 8 contiguous mini rows per wave, first 3 stages
    T a[8][8];
    {
        const int tr0 = wave * 8;
        const int t = tr0 >> G;
        const int mu = rt * NMINI + t;
        const int B = mu >> j0;
        const int u = mu & ((1 << j0) - 1);
        const bool active = (mu < n_mini) && ((u << G) <= d.row_limit);
        if (!active) {
#pragma unroll
            for (int r = 0; r < 8; ++r) zero8(a[r]);
        } else if (FIRST && d.src_kind == SRC_IMAGE_T && d.S1 == 0) {
            // first pass (u = 0): the wave's rows are 8 consecutive image columns
            load_rows_transposed<TIn, T>(d, (B << G) + (tr0 & ((1 << G) - 1)), xw0, lane, a);
        } else {
            int e0[8];
            bool patch[8];
            bool any = false;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int m = (tr0 + r) & ((1 << G) - 1);
                const int R = (B << (j0 + G)) + (m << j0) + u;
                if constexpr (FIRST) {
                    patch[r] = d.src_kind == SRC_IMAGE ? issue_image_row<TIn, T>(d, R, xw0, lane, a[r], e0[r])
                                                       : issue_image_t_row<TIn, T>(d, R, xw0, lane, a[r], e0[r]);
                } else {
                    patch[r] = issue_band_row<T>(d, R, xw0 + DIR * u * m, lane, a[r], e0[r]);
                }
                any |= patch[r];
            }
            if (__any(any)) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    if (patch[r]) {
                        const int m = (tr0 + r) & ((1 << G) - 1);
                        const int R = (B << (j0 + G)) + (m << j0) + u;
                        if constexpr (FIRST) patch_image_row<TIn, T>(d, R, e0[r], a[r]);
                        else patch_band_row<T>(d, R, e0[r], a[r]);
                    }
                }
            }
        }
    }
    fwd_stage<T, DIR, 0>(a);
    fwd_stage<T, DIR, 1>(a);
    fwd_stage<T, DIR, 2>(a);

    // ---- phase B: rows 8g + u' with offsets dir*u'*g, last GB stages.  The
    // exchange runs in two halves (registers 0-3, then 4-7 of every wave) so
    // the LDS holds 32 rows and two workgroups fit on a CU.
    T b[8][8];
    if constexpr (GB == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < 8; ++c) b[r][c] = a[r][c];
    } else {
        const int my_half = ((wave << (3 - GB)) & 7) >> 2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            {
                // column 8*lane + c + LOFF of LDS row wave*4 + rr: plane c, slot lane + LOFF/8
                T* lw = lds + wave * 4 * kLdsRow + lane + LOFF / 8;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                    for (int c = 0; c < 8; ++c) lw[rr * kLdsRow + c * kPlane] = a[4 * h + rr][c];
            }
            __syncthreads();
            if (my_half == h) {
#pragma unroll
                for (int rho = 0; rho < 8; ++rho) {
                    const int rp = rho & ((1 << GB) - 1);
                    const int q = rho >> GB;
                    const int kappa = (wave << (3 - GB)) + q;
                    const int t = kappa >> 3;
                    const int up = kappa & 7;
                    const int wa = (t << GB) + rp;         // phase-A wave holding the row
                    const int off = uniform(DIR * up * rp + LOFF);
                    lds_read8<T>(lds + (wa * 4 + (up & 3)) * kLdsRow + lane, off, b[rho]);
                }
            }
            if (h == 0) __syncthreads();
        }
    }
    fwd_stages_b<T, DIR, GB>(b);

    // ---- store
    const int wc0 = 8 * lane;
    const bool lane_ok = DIR > 0 ? (wc0 < VW) : (wc0 >= (1 << G));
    if (!lane_ok) return;
    const int x0 = xw0 + wc0;
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
        if constexpr (!LAST) {
            T* dst = reinterpret_cast<T*>(d.dst) + (long long)out_row * d.dst_ld;
            const int e0 = x0 + d.dst_off;
            if (e0 + 8 <= d.dst_bw) {
                store8<T>(dst + e0, b[rho]);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (e0 + c < d.dst_bw) dst[e0 + c] = b[rho][c];
            }
        } else {
            const int s = out_row;
            if (s == d.skip_row) continue;
            T* dst = reinterpret_cast<T*>(d.dst) + (long long)(d.row_base + d.row_sign * s) * d.dst_ld;
            const int roll = d.shifted ? ((d.roll_a + d.roll_b * s) >> 1) : 0;
            const int W = d.W;
            if (x0 >= W) continue;
            const int xr = wrap_lane(x0 + roll, W);
            if (x0 + 8 <= W && xr + 8 <= W) {
                store8_stream<T>(dst + xr, b[rho]);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (x0 + c < W) {
                        int e = xr + c;
                        if (e >= W) e -= W;
                        dst[e] = b[rho][c];
                    }
                }
            }
        }
    }
}

template <typename TIn, typename T, int GB, bool FIRST, bool LAST>
__global__ __launch_bounds__(kThreads, 4) void fht_pass_kernel(const PassLaunch L)
{
    __shared__ T lds[kTileRows / 2 * kLdsRow];
    const PassDesc& d = L.d[blockIdx.z];
    if ((int)blockIdx.x >= d.n_windows || (int)blockIdx.y >= d.n_row_tiles) return;
    if (d.dir > 0) fwd_tile<TIn, T, GB, 1, FIRST, LAST>(d, blockIdx.y, blockIdx.x, lds);
    else fwd_tile<TIn, T, GB, -1, FIRST, LAST>(d, blockIdx.y, blockIdx.x, lds);
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

// Source row of an adjoint pass (Hough gradient or band), issue + patch as
// for the forward loads.
template <typename T, bool FROM_HOUGH>
__device__ __forceinline__ bool adj_issue_row(const AdjDesc& d, int s_row, int xrow, int lane, T (&v)[8], int& e0)
{
    const int W = d.W;
    if constexpr (!FROM_HOUGH) {
        const T* band = reinterpret_cast<const T*>(d.src) + (long long)s_row * d.src_ld;
        e0 = wrap_lane(mod_w(xrow + d.src_off, W) + 8 * lane, W);
        const bool fast = e0 + 8 <= d.src_bw;
        const bool zero = e0 >= d.src_bw && e0 + 8 <= W;
        load8<T>(fast ? band + e0 : zero_page<T>(), v);
        return !fast && !zero;
    } else {
        const bool skip = s_row == d.skip_row;
        const T* src = reinterpret_cast<const T*>(d.src) + (long long)(d.row_base + d.row_sign * s_row) * d.src_ld;
        const int roll = d.shifted ? ((d.roll_a + d.roll_b * s_row) >> 1) : 0;
        e0 = wrap_lane(mod_w(xrow + roll, W) + 8 * lane, W);
        const bool fast = !skip && e0 + 8 <= W;
        load8<T>(fast ? src + e0 : zero_page<T>(), v);
        return !skip && !fast;
    }
}

template <typename T, bool FROM_HOUGH>
__device__ __forceinline__ void adj_patch_row(const AdjDesc& d, int s_row, int e0, T (&v)[8])
{
    const int W = d.W;
    if constexpr (!FROM_HOUGH) {
        const T* band = reinterpret_cast<const T*>(d.src) + (long long)s_row * d.src_ld;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            int e = e0 + c;
            if (e >= W) e -= W;
            v[c] = (e < d.src_bw) ? band[e] : (T)0;
        }
    } else {
        const T* src = reinterpret_cast<const T*>(d.src) + (long long)(d.row_base + d.row_sign * s_row) * d.src_ld;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            int e = e0 + c;
            if (e >= W) e -= W;
            v[c] = src[e];
        }
    }
}

template <typename T>
__device__ __forceinline__ void acc_store8(T* p, const T (&v)[8], bool accumulate)
{
    if (accumulate) {
        T o[8];
        load8<T>(p, o);
        T s[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) s[c] = o[c] + v[c];
        store8<T>(p, s);
    } else {
        store8<T>(p, v);
    }
}

template <typename T, int GB, int DIR, bool FIRST, bool LAST>
__device__ __forceinline__ void adj_tile(const AdjDesc& d, int rt, int win, T* lds)
{
    constexpr int G = 3 + GB;
    constexpr int NMINI = 1 << (6 - G);
    constexpr int VW = kWinCols - (1 << G);
    // transposed shifts point the other way, so the halo sits on the other side
    constexpr int LOFF = DIR > 0 ? 0 : kLdsOffNeg;
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    const int j0 = d.j0;
    const int n_mini = d.n >> G;
    const int x_lo = d.x_start + win * VW;
    const int xw0 = x_lo - (DIR > 0 ? (1 << G) : 0);

    // ---- load the forward pass's output rows (contiguous within a block)
    T b[8][8];
    {
        int e0[8];
        bool patch[8];
        bool any = false;
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
                patch[rho] = adj_issue_row<T, FIRST>(d, s_row, xw0, lane, b[rho], e0[rho]);
            } else {
                zero8(b[rho]);
                patch[rho] = false;
                e0[rho] = 0;
            }
            any |= patch[rho];
        }
        if (__any(any)) {
#pragma unroll
            for (int rho = 0; rho < 8; ++rho) {
                if (patch[rho]) {
                    const int rp = rho & ((1 << GB) - 1);
                    const int q = rho >> GB;
                    const int kappa = (wave << (3 - GB)) + q;
                    const int t = kappa >> 3;
                    const int up = kappa & 7;
                    const int mu = rt * NMINI + t;
                    const int B = mu >> j0;
                    const int u = mu & ((1 << j0) - 1);
                    const int s_row = (B << (j0 + G)) + (u << G) + (up << GB) + rp;
                    adj_patch_row<T, FIRST>(d, s_row, e0[rho], b[rho]);
                }
            }
        }
    }
    adj_stages_b<T, DIR, GB>(b);

    // ---- exchange (two halves of LDS rows, as in the forward pass)
    T a[8][8];
    if constexpr (GB == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int c = 0; c < 8; ++c) a[r][c] = b[r][c];
    } else {
        const int my_half = ((wave << (3 - GB)) & 7) >> 2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (my_half == h) {
#pragma unroll
                for (int rho = 0; rho < 8; ++rho) {
                    const int rp = rho & ((1 << GB) - 1);
                    const int q = rho >> GB;
                    const int kappa = (wave << (3 - GB)) + q;
                    const int t = kappa >> 3;
                    const int up = kappa & 7;
                    const int wa = (t << GB) + rp;
                    const int off = uniform(DIR * up * rp + LOFF);
                    lds_write8<T>(lds + (wa * 4 + (up & 3)) * kLdsRow + lane, off, b[rho]);
                }
            }
            __syncthreads();
            {
                const T* lr = lds + wave * 4 * kLdsRow + lane + LOFF / 8;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                    for (int c = 0; c < 8; ++c) a[4 * h + rr][c] = lr[rr * kLdsRow + c * kPlane];
            }
            if (h == 0) __syncthreads();
        }
    }
    adj_stage<T, DIR, 2>(a);
    adj_stage<T, DIR, 1>(a);
    adj_stage<T, DIR, 0>(a);

    // ---- store row m of each mini transform at its offset dir*u*m
    const int wc0 = 8 * lane;
    const bool lane_ok = DIR > 0 ? (wc0 >= (1 << G)) : (wc0 < VW);
    if (!lane_ok) return;
    const int x0 = xw0 + wc0;  // window column of register 0 (before the offset)
    const int W = d.W;
    const int tr0 = wave * 8;
    const int t = tr0 >> G;
    const int mu = rt * NMINI + t;
    if (mu >= n_mini) return;
    const int B = mu >> j0;
    const int u = mu & ((1 << j0) - 1);
    if constexpr (!LAST) {
        // band: window columns [0, W) are covered once; column z of row m lands
        // on z + dir*u*m, a bijection of the cyclic row
        if (x0 >= W) return;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int m = (tr0 + r) & ((1 << G) - 1);
            const int R = (B << (j0 + G)) + (m << j0) + u;
            T* dst = reinterpret_cast<T*>(d.dst) + (long long)R * d.dst_ld;
            const int e0 = wrap_lane(mod_w(xw0 + DIR * u * m + d.dst_off, W) + wc0, W);
            if (x0 + 8 <= W && e0 + 8 <= d.dst_bw) {
                store8<T>(dst + e0, a[r]);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (x0 + c < W) {
                        int e = e0 + c;
                        if (e >= W) e -= W;
                        if (e < d.dst_bw) dst[e] = a[r][c];
                    }
                }
            }
        }
    } else if (d.dst_kind == 1) {
        // image rows (the first forward pass has u = 0: no offset remains)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int R = (B << G) + ((tr0 + r) & ((1 << G) - 1));
            if (R >= d.img_h || x0 >= d.img_w) continue;
            T* p = reinterpret_cast<T*>(d.dst) + (long long)R * d.dst_ld + x0;
            if (x0 + 8 <= d.img_w) {
                acc_store8<T>(p, a[r], d.accumulate != 0);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (x0 + c < d.img_w) p[c] = d.accumulate ? (T)(p[c] + a[r][c]) : a[r][c];
            }
        }
    } else {
        // transposed image: rows R0..R0+7 are image columns, contiguous in memory
        const int R0 = (B << G) + (tr0 & ((1 << G) - 1));
        const bool all_cols = R0 + 8 <= d.img_w;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int e = x0 + c;  // image row
            if (e >= d.img_h) continue;
            T* p = reinterpret_cast<T*>(d.dst) + (long long)e * d.dst_ld + R0;
            T v[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) v[r] = a[r][c];
            if (all_cols) {
                acc_store8<T>(p, v, d.accumulate != 0);
            } else {
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (R0 + r < d.img_w) p[r] = d.accumulate ? (T)(p[r] + v[r]) : v[r];
            }
        }
    }
}

template <typename T, int GB, bool FIRST, bool LAST>
__global__ __launch_bounds__(kThreads, 4) void fht_adj_pass_kernel(const AdjLaunch L)
{
    __shared__ T lds[kTileRows / 2 * kLdsRow];
    const AdjDesc& d = L.d[blockIdx.z];
    if ((int)blockIdx.x >= d.n_windows || (int)blockIdx.y >= d.n_row_tiles) return;
    if (d.dir > 0) adj_tile<T, GB, 1, FIRST, LAST>(d, blockIdx.y, blockIdx.x, lds);
    else adj_tile<T, GB, -1, FIRST, LAST>(d, blockIdx.y, blockIdx.x, lds);
}

// Adjoint for n <= 4 rows: B_j from B_{j+1} by the transposed stage, top-down.
template <typename T, int J, int K>
__device__ T adj_direct(const AdjDesc& d, int row, int x)
{
    if constexpr (J == K) {
        T v[8];
        int e0;
        if (adj_issue_row<T, true>(d, row, x, 0, v, e0)) adj_patch_row<T, true>(d, row, e0, v);
        return v[0];  // only the first column is used
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
