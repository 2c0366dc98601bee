// Device code of the dyadic Fast Hough Transform for gfx950 (CDNA4): the
// kernel templates, instantiated per element type in fht_fwd_*.hip and
// fht_adj_*.hip.
//
// The transform of one quadrant is the stage recurrence of Brady's FHT
// (arXiv 1811.06378, section 2 and section 4 / Fig. 6): after stage j the rows
// form blocks of 2^(j+1); stage j merges two neighbouring blocks,
//   A[j+1][b*2^(j+1) + t][xi] = A[j][b*2^(j+1) + (t>>1)][xi]
//                             + A[j][b*2^(j+1) + 2^j + (t>>1)][xi + (t - (t>>1))]   (mod W),
// written in the quadrant's column coordinate xi = dir * x, in which every
// quadrant's patterns lean the same way (quadrants 2 and 3 are mirrored).
//
// Stage fusion.  G consecutive stages starting at stage j0 regroup exactly:
// with u < 2^j0, m, v < 2^G,
//   A[j0+G][B*2^(j0+G) + u*2^G + v][xi]
//     = MiniFHT_G( m -> A[j0][B*2^(j0+G) + m*2^j0 + u][xi + u*m] )[v][xi],
// i.e. the same G-stage transform on the 2^G rows m*2^j0 + u, each read with a
// per-row column offset u*m.  Applied twice inside a tile (G = 3 + GB): the
// first 3 stages run on 8 contiguous rows held by one wave, the last GB stages
// on rows 8g + u' read back from LDS with offsets u'*g.
//
// Register layout.  A workgroup (8 waves) holds 64 rows x 512 columns; a lane
// owns 8 consecutive columns of 8 rows.  A stage's column shift (at most 4 in
// registers) reads the lane's own registers or, across the lane boundary, the
// next lane's registers through a DPP wavefront shift by one lane, so the
// shift costs no LDS traffic.  The last 2^G - 1 columns of a tile are halo:
// computed, not stored.
//
// No MFMA: the recurrence is a bandwidth-bound chain of additions.
#pragma once

#include "fht_internal.h"

#include <climits>

namespace fht {

// ------------------------------------------------------------ small helpers

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

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Storage row of quadrant row R in an intermediate band written after j of
// the k stages.  Row R = (b << j) + v (block b, row v of the block) is stored
// at (v << (k - j)) + b: the next pass reads rows (m << j) + u for 2^G
// consecutive m, which land on consecutive storage rows (one contiguous run
// instead of rows 2^j apart).  Writer and reader use the same j.
__device__ __forceinline__ int band_row(int R, int j, int k)
{
    return ((R & ((1 << j) - 1)) << (k - j)) + (R >> j);
}

// a mod W for a wave-uniform a (|a| < 4W whenever W >= 1024 in the pass
// geometry; small W takes the division).
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
__device__ __forceinline__ int wrap_up(int e, int W)
{
    if (e >= W) e -= W;
    if (e >= W) e %= W;
    return e;
}

// e in (-512, W) -> e mod W
__device__ __forceinline__ int wrap_down(int e, int W)
{
    if (e < 0) e += W;
    if (e < 0) e = mod_pos(e, W);
    return e;
}

// Memory start of the lane's 8-column run.  The lane's registers c = 0..7 hold
// xi = xi0 + 8*lane + c.  Unmirrored, column x = xi + shift_x and the run
// ascends from x(c=0); mirrored, x = -xi + shift_x, so register c sits at
// run_start + 7 - c.
__device__ __forceinline__ int lane_run_start(int xi0, int shift_x, int lane, int W, int mirror)
{
    if (!mirror) return wrap_up(mod_w(xi0 + shift_x, W) + 8 * lane, W);
    return wrap_down(mod_w(-xi0 - 7 + shift_x, W) - 8 * lane, W);
}

// Column of register c for a run start (element patch paths).
__device__ __forceinline__ int run_col(int start, int c, int W, int mirror)
{
    int e = start + (mirror ? 7 - c : c);
    return e >= W ? e - W : e;
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

template <typename T>
__device__ __forceinline__ void reverse8(T (&v)[8])
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const T t = v[c];
        v[c] = v[7 - c];
        v[7 - c] = t;
    }
}

// 8 consecutive source elements.  For bytes at any address: the two aligned
// dwords from the dword holding p[0], plus the dword holding p[7] when p is
// not dword-aligned (else that dword again), funnel-shifted by the byte
// offset.  Every dword read holds at least one of the 8 wanted bytes, so no
// read reaches a page the wanted bytes do not touch.
template <typename TIn, typename T>
__device__ __forceinline__ void load8_src(const TIn* p, T (&v)[8])
{
    if constexpr (sizeof(TIn) == 1) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(p);
        const uint32_t* base = reinterpret_cast<const uint32_t*>(a & ~(uintptr_t)3);
        const uint32_t sh = (uint32_t)(a & 3) * 8u;
        const u32x2u w = *reinterpret_cast<const u32x2u*>(base);
        const uint32_t w2 = base[sh ? 2 : 1];
        const uint32_t lo = __builtin_amdgcn_alignbit(w.y, w.x, sh);
        const uint32_t hi = __builtin_amdgcn_alignbit(w2, w.y, sh);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v[c] = (T)((lo >> (8 * c)) & 0xFFu);
            v[4 + c] = (T)((hi >> (8 * c)) & 0xFFu);
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

// Loads are issued for all rows before any result is used: lanes whose 8
// columns lie inside the data read them with 16-byte loads, lanes whose 8
// columns are all zero padding read a static zero page, and only lanes that
// straddle a boundary (rare) are patched element by element afterwards.  An
// if/else per row would make every row wait for the previous row's loads.
static __device__ __attribute__((aligned(64))) unsigned int g_zero_page[16];

template <typename T>
__device__ __forceinline__ const T* zero_page()
{
    return reinterpret_cast<const T*>(g_zero_page);
}

// --------------------------------------------------------- register stages

// Forward stage J on 8 register rows: blocks of 2^(J+1) rows; block rows 2i
// and 2i+1 both come from the pair (top row i, bottom row 2^J + i), the
// bottom one shifted by i and i+1 columns.  Each output pair depends on one
// input pair only: the stage is a set of row butterflies.
// The operation along the patterns: 0 = sum (the transform), 1 = max (the
// same patterns under another associative, commutative operation, section 1).
template <int OP, typename T>
__device__ __forceinline__ T combine(T x, T y)
{
    if constexpr (OP == 0) return x + y;
    else if constexpr (sizeof(T) == 4 && T(0.5) != T(0)) return __builtin_fmaxf(x, y);
    else return x > y ? x : y;
}

template <typename T, int J, int OP = 0>
__device__ __forceinline__ void fwd_stage(T (&a)[8][8])
{
    constexpr int H = 1 << J;
    T o[8][8];
#pragma unroll
    for (int blk = 0; blk < 8; blk += 2 * H) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int c0 = c + i, c1 = c + i + 1;
                const T b0 = c0 >= 8 ? dpp_move<kDppFromNext>(a[blk + H + i][c0 - 8]) : a[blk + H + i][c0];
                const T b1 = c1 >= 8 ? dpp_move<kDppFromNext>(a[blk + H + i][c1 - 8]) : a[blk + H + i][c1];
                o[blk + 2 * i][c] = combine<OP>(a[blk + i][c], b0);
                o[blk + 2 * i + 1][c] = combine<OP>(a[blk + i][c], b1);
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
//   top[i][xi]    = g[2i][xi] + g[2i+1][xi]
//   bottom[u][xi] = g[2u][xi - u] + g[2u+1][xi - u - 1].
template <typename T, int J>
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
                const int c0 = c - u, c1 = c - u - 1;
                const T x0 = c0 < 0 ? dpp_move<kDppFromPrev>(a[blk + 2 * u][c0 + 8]) : a[blk + 2 * u][c0];
                const T x1 = c1 < 0 ? dpp_move<kDppFromPrev>(a[blk + 2 * u + 1][c1 + 8]) : a[blk + 2 * u + 1][c1];
                o[blk + H + u][c] = x0 + x1;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) a[r][c] = o[r][c];
}

template <typename T, int GB, int OP = 0>
__device__ __forceinline__ void fwd_stages_b(T (&b)[8][8])
{
    if constexpr (GB > 0) fwd_stage<T, 0, OP>(b);
    if constexpr (GB > 1) fwd_stage<T, 1, OP>(b);
    if constexpr (GB > 2) fwd_stage<T, 2, OP>(b);
}

template <typename T, int GB>
__device__ __forceinline__ void adj_stages_b(T (&b)[8][8])
{
    if constexpr (GB > 2) adj_stage<T, 2>(b);
    if constexpr (GB > 1) adj_stage<T, 1>(b);
    if constexpr (GB > 0) adj_stage<T, 0>(b);
}

// ------------------------------------------------------------------ LDS

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

// For the writes (the adjoint's exchange), the empty asm statements,
// distinct per residue, keep the compiler from merging the 8 cases into one
// with per-element address arithmetic (seven adds and address registers
// per row); kept apart, the first adjoint pass of 4096^2 f32 is about 4 us
// faster.  The same for the reads made the forward's first pass 4 us
// slower, so they are left to the compiler.
template <int O7, typename T>
__device__ __forceinline__ void lds_write8_fixed(T* p, const T (&v)[8])
{
    asm volatile("; lds row write, residue %0" ::"n"(O7));
#pragma unroll
    for (int c = 0; c < 8; ++c) p[((c + O7) & 7) * kPlane + ((c + O7) >> 3)] = v[c];
    asm volatile("; lds row write, residue %0, issued" ::"n"(O7));
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

// ------------------------------------------------------------ source loads

// Band row at xi = xrow + 8*lane + c (band index = (xi + src_off) mod W).
template <typename T>
__device__ __forceinline__ bool issue_band_row(const T* row_ptr, int src_off, int src_bw, int W, int xrow, int lane,
                                               T (&v)[8], int& e0)
{
    e0 = wrap_up(mod_w(xrow + src_off, W) + 8 * lane, W);
    const bool fast = e0 + 8 <= src_bw;
    const bool zero = e0 >= src_bw && e0 + 8 <= W;
    load8<T>(fast ? row_ptr + e0 : zero_page<T>(), v);
    return !fast && !zero;
}

template <typename T>
__device__ __forceinline__ void patch_band_row(const T* row_ptr, int src_bw, int W, int e0, T (&v)[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        int e = e0 + c;
        if (e >= W) e -= W;
        v[c] = (e < src_bw) ? row_ptr[e] : (T)0;
    }
}

// Image row R of quadrants 1, 2 (x = +-xi, sheared for the angle range).
// The 8 values arrive in memory order; a mirrored row is reversed by the
// caller once every row's loads are issued (reversing here, behind the
// runtime mirror flag, made each row wait for its own loads before the next
// row's were issued).
template <typename TIn, typename T>
__device__ __forceinline__ bool issue_image_row(const PassDesc& d, int R, int xrow, int lane, T (&v)[8], int& e0)
{
    const int W = d.W;
    const TIn* p = reinterpret_cast<const TIn*>(d.src) + (long long)R * d.src_ld;
    e0 = lane_run_start(xrow, -shear_of_row(R, d.S1, d.n), lane, W, d.mirror);
    const bool row_ok = R < d.img_h;
    const bool fast = row_ok && e0 + 8 <= d.img_w;
    const bool zero = !row_ok || (e0 >= d.img_w && e0 + 8 <= W);
    load8_src<TIn, T>(fast ? p + e0 : zero_page<TIn>(), v);
    return !fast && !zero;
}

// Element loads of one source row.  With a scale (section 4), column e of
// the scaled image (extent img_w or img_h along the sheared axis) is source
// sample floor(e * den / num).
template <typename TIn, typename T>
__device__ __forceinline__ void patch_image_row(const PassDesc& d, int R, int e0, T (&v)[8])
{
    const TIn* img = reinterpret_cast<const TIn*>(d.src);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int e = run_col(e0, c, d.W, d.mirror);
        const int es = d.scale_num ? (int)(((long long)e * d.scale_den) / d.scale_num) : e;
        if (d.src_kind == SRC_IMAGE)
            v[c] = (R < d.img_h && e < d.img_w) ? to_acc<T>(img[(long long)R * d.src_ld + es]) : (T)0;
        else
            v[c] = (R < d.img_w && e < d.img_h) ? to_acc<T>(img[(long long)es * d.src_ld + R]) : (T)0;
    }
}

// Element loads of unsheared, unscaled image row R at the run starting at
// column e0 (boundary lanes of the first pass).
template <typename TIn, typename T>
__device__ __forceinline__ void patch_image_row_plain(const PassDesc& d, int R, int e0, T (&v)[8])
{
    const TIn* row = reinterpret_cast<const TIn*>(d.src) + (long long)R * d.src_ld;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int e = run_col(e0, c, d.W, d.mirror);
        v[c] = (R < d.img_h && e < d.img_w) ? to_acc<T>(row[e]) : (T)0;
    }
}

// Element-load rows (transposed image with a shear, or a scaled source):
// zeros now, every element loaded by patch_image_row.
template <typename TIn, typename T>
__device__ __forceinline__ bool issue_image_t_row(const PassDesc& d, int R, int xrow, int lane, T (&v)[8], int& e0)
{
    e0 = lane_run_start(xrow, -shear_of_row(R, d.S1, d.n), lane, d.W, d.mirror);
    zero8(v);
    return true;
}

// Rows R0..R0+7 of the transposed image (image columns), unsheared: for each
// of the lane's 8 columns (image rows) the 8 values are contiguous in memory.
template <typename TIn, typename T>
__device__ __forceinline__ void load_rows_transposed(const PassDesc& d, int R0, int xrow, int lane, T (&a)[8][8])
{
    const int W = d.W;
    const int e0 = lane_run_start(xrow, 0, lane, W, d.mirror);
    const TIn* img = reinterpret_cast<const TIn*>(d.src);
    const bool all_cols = R0 + 8 <= d.img_w;
    unsigned patch = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int e = run_col(e0, c, W, d.mirror);
        const TIn* p = img + (long long)e * d.src_ld + R0;
        const bool inside = e < d.img_h;
        const bool fast = inside && all_cols;
        T t[8];
        load8_src<TIn, T>(fast ? p : zero_page<TIn>(), t);
#pragma unroll
        for (int r = 0; r < 8; ++r) a[r][c] = t[r];
        if (inside && !fast) patch |= 1u << c;
    }
    if (__any(patch != 0)) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (patch & (1u << c)) {
                const int e = run_col(e0, c, W, d.mirror);
                const TIn* p = img + (long long)e * d.src_ld + R0;
#pragma unroll
                for (int r = 0; r < 8; ++r) a[r][c] = (R0 + r < d.img_w) ? to_acc<T>(p[r]) : (T)0;
            }
        }
    }
}

// ------------------------------------------------------ fused forward pass

// Phase B of a forward tile for GB = G - 3 stages after the exchange.  The
// exchange runs in two halves (registers 0-3, then 4-7 of every wave) so the
// LDS holds 32 rows and two workgroups fit on a CU.
template <typename T, int GB, int OP = 0>
__device__ __forceinline__ void fwd_phase_b(T (&a)[8][8], T (&b)[8][8], T* lds, int wave, int lane)
{
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
                // column 8*lane + c of LDS row wave*4 + rr: plane c, slot lane
                T* lw = lds + wave * 4 * kLdsRow + lane;
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
                    const int wa = (t << GB) + rp;  // phase-A wave holding the row
                    lds_read8<T>(lds + (wa * 4 + (up & 3)) * kLdsRow + lane, uniform(up * rp), b[rho]);
                }
            }
            if (h == 0) __syncthreads();
        }
        fwd_stages_b<T, GB, OP>(b);
    }
}

// Stores of one forward tile: rows of b to the band of the pass, or (last
// pass) to the Hough image with the merged-row mapping, the mirror and the
// optional fhtshift roll.
template <typename T, int GB, bool LAST, int NW>
__device__ __forceinline__ void fwd_store(const PassDesc& d, int rt, int xi0, int wave, int lane, const T (&b)[8][8])
{
    constexpr int G = 3 + GB;
    constexpr int VW = kWinCols - (1 << G);
    constexpr int NMINI = (NW * 8) >> G;
    const int j0 = d.j0;
    const int n_mini = d.n >> G;
    const int wc0 = 8 * lane;
    if (wc0 >= VW) return;
    const int xi = xi0 + wc0;  // xi of register 0
    const int W = d.W;
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
            const int k = 31 - __builtin_clz(d.n);
            T* dst = reinterpret_cast<T*>(d.dst) + (long long)band_row(out_row, j0 + G, k) * d.dst_ld;
            const int e0 = xi + d.dst_off;
            if (e0 + 8 <= d.dst_bw) {
                store8<T>(dst + e0, b[rho]);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (e0 + c < d.dst_bw) dst[e0 + c] = b[rho][c];
            }
        } else {
            const int s = out_row;
            const int rel = xi - d.x_start;  // 0..W-1 over the windows
            if (s == d.skip_row || rel >= W) continue;
            T* dst = reinterpret_cast<T*>(d.dst) + (long long)(d.row_base + d.row_sign * s) * d.dst_ld;
            const int roll = d.shifted ? ((d.roll_a + d.roll_b * s) >> 1) : 0;
            // memory run of the lane's 8 columns (descending for mirrored quadrants)
            const int e0 = d.mirror ? wrap_down(mod_w(-xi - 7 + roll, W), W) : wrap_up(mod_w(xi + roll, W), W);
            if (rel + 8 <= W && e0 + 8 <= W) {
                T v[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) v[c] = d.mirror ? b[rho][7 - c] : b[rho][c];
                store8<T>(dst + e0, v);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (rel + c < W) dst[run_col(e0, c, W, d.mirror)] = b[rho][c];
            }
        }
    }
}


// One tile (NW * 8 rows x 512 columns: NW waves of 8 rows) of one forward
// pass of G = 3 + GB stages.  rt: row tile, win: column window.  Every thread
// of the workgroup calls it; lds holds NW * 4 rows of kLdsRow words.
// SRCM, the first pass's image sources: 0 unsheared rows or the transposed
// image; 1 rows sheared for the angle range; 2 element loads (scaled sources,
// sheared transposed sources).  Each kernel holds only its own source path:
// the element path alone is about 80 KB of code, and with every path in one
// kernel the instruction fetches delayed every tile of small transforms.
template <typename TIn, typename T, int GB, bool FIRST, bool LAST, int OP = 0, int NW = 8, int SRCM = 0>
__device__ __forceinline__ void fwd_tile(const PassDesc& d, int rt, int win, T* lds)
{
    constexpr int G = 3 + GB;
    constexpr int ROWS = NW * 8;
    static_assert(ROWS >= (1 << G), "a tile holds whole mini-transforms");
    constexpr int VW = kWinCols - (1 << G);      // stored columns per tile
    constexpr int NMINI = ROWS >> G;             // mini-transforms of 2^G rows per tile
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    const int j0 = d.j0;
    const int n_mini = d.n >> G;                 // mini-transforms in the quadrant
    const int k = 31 - __builtin_clz(d.n);       // stages of the quadrant
    const int xi0 = d.x_start + win * VW;        // xi of the tile's column 0

    // A last-pass tile lying wholly in the black zone of every one of its rows
    // (section 3.2, case c) is written as zeros without loading anything.
    bool black = false;
    if (LAST && d.black_ok) {
        const int s_max = min(rt * ROWS + ROWS - 1, d.n - 1);
        black = xi0 >= d.black_lo && xi0 + VW <= d.black_lo + d.n - s_max;
    }

    T b[8][8];
    if (black) {
#pragma unroll
        for (int r = 0; r < 8; ++r) zero8(b[r]);
    } else {
        // ---- phase A: 8 contiguous mini rows per wave, first 3 stages
        T a[8][8];
        const int tr0 = wave * 8;
        const int t = tr0 >> G;
        const int mu = rt * NMINI + t;
        const int B = mu >> j0;
        const int u = mu & ((1 << j0) - 1);
        const bool active = (mu < n_mini) && ((u << G) <= d.row_limit);
        // Raised issue priority while this wave issues its loads, so that
        // they go out ahead of the other resident workgroup's arithmetic
        // (measured: last pass of 4096^2 f32 about 2% faster; raising it
        // for the stores as well gained nothing).
        __builtin_amdgcn_s_setprio(2);
        if (!active) {
#pragma unroll
            for (int r = 0; r < 8; ++r) zero8(a[r]);
        } else if constexpr (FIRST && SRCM == 0) {
            if (d.src_kind == SRC_IMAGE_T) {
                // the wave's rows are 8 consecutive image columns (u = 0)
                load_rows_transposed<TIn, T>(d, (B << G) + (tr0 & ((1 << G) - 1)), xi0, lane, a);
            } else {
                // the wave's 8 rows are consecutive image rows read at the
                // same columns, so the lane's column run is computed once;
                // every row's loads are issued before the first wait
                const int R0 = (B << G) + (tr0 & ((1 << G) - 1));
                const int ec = lane_run_start(xi0, 0, lane, d.W, d.mirror);
                const bool col_fast = ec + 8 <= d.img_w;
                const bool col_zero = ec >= d.img_w && ec + 8 <= d.W;
                const TIn* p = reinterpret_cast<const TIn*>(d.src) + (long long)R0 * d.src_ld + ec;
                bool patch[8];
                bool any = false;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const bool row_ok = R0 + r < d.img_h;
                    const bool fast = row_ok && col_fast;
                    load8_src<TIn, T>(fast ? p + (long long)r * d.src_ld : zero_page<TIn>(), a[r]);
                    patch[r] = row_ok && !col_fast && !col_zero;
                    any |= patch[r];
                }
                if (d.mirror) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) reverse8(a[r]);
                }
                if (__any(any)) {
#pragma unroll
                    for (int r = 0; r < 8; ++r)
                        if (patch[r]) patch_image_row_plain<TIn, T>(d, R0 + r, ec, a[r]);
                }
            }
        } else {
            int e0[8];
            bool patch[8];
            bool any = false;
            const T* band = reinterpret_cast<const T*>(d.src);
            // The source kind is chosen once for all rows: a choice per row
            // ends every row in a merge of two paths, where the register
            // moves wait for that row's loads before the next row's issue.
            if constexpr (!FIRST || SRCM == 1) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int m = (tr0 + r) & ((1 << G) - 1);
                    const int R = (B << (j0 + G)) + (m << j0) + u;
                    if constexpr (FIRST)
                        patch[r] = issue_image_row<TIn, T>(d, R, xi0, lane, a[r], e0[r]);
                    else
                        patch[r] = issue_band_row<T>(band + (long long)band_row(R, j0, k) * d.src_ld, d.src_off,
                                                     d.src_bw, d.W, xi0 + u * m, lane, a[r], e0[r]);
                    any |= patch[r];
                }
                if (FIRST && d.mirror) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) reverse8(a[r]);
                }
            } else {
                // transposed sheared or scaled sources: the element path
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int m = (tr0 + r) & ((1 << G) - 1);
                    const int R = (B << (j0 + G)) + (m << j0) + u;
                    patch[r] = issue_image_t_row<TIn, T>(d, R, xi0, lane, a[r], e0[r]);
                    any |= patch[r];
                }
            }
            if (__any(any)) {
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    if (patch[r]) {
                        const int m = (tr0 + r) & ((1 << G) - 1);
                        const int R = (B << (j0 + G)) + (m << j0) + u;
                        if constexpr (FIRST && SRCM == 1) patch_image_row_plain<TIn, T>(d, R, e0[r], a[r]);
                        else if constexpr (FIRST) patch_image_row<TIn, T>(d, R, e0[r], a[r]);
                        else patch_band_row<T>(band + (long long)band_row(R, j0, k) * d.src_ld, d.src_bw, d.W, e0[r],
                                               a[r]);
                    }
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
        fwd_stage<T, 0, OP>(a);
        fwd_stage<T, 1, OP>(a);
        fwd_stage<T, 2, OP>(a);
        // ---- phase B: rows 8g + u' read with offsets u'*g, last GB stages
        fwd_phase_b<T, GB, OP>(a, b, lds, wave, lane);
    }

    fwd_store<T, GB, LAST, NW>(d, rt, xi0, wave, lane, b);
}

// Tile order.  Workgroups are dispatched to the 8 XCDs round-robin by block
// index; numbering the tiles so that each XCD receives a contiguous run of
// them keeps neighbouring windows (which share 2^G - 1 halo columns) and
// neighbouring row tiles in one L2.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_tile(int block, int n_tiles)
{
    const int per = (n_tiles + kXcds - 1) / kXcds;
    return (block % kXcds) * per + block / kXcds;
}

// NW = 8: 64-row tiles, two workgroups per CU; NW = 4: 32-row tiles (passes
// of at most 5 stages), half the LDS, four workgroups per CU.
template <typename TIn, typename T, int GB, bool FIRST, bool LAST, int OP, int NW, int SRCM>
__global__ __launch_bounds__(NW * 64, 4) void fht_pass_kernel(const PassLaunch L)
{
    __shared__ T lds[NW * 4 * kLdsRow];
    int t = xcd_tile(blockIdx.x, L.n_tiles);
    if (t >= L.n_tiles) return;
    int z = 0;
    while (z + 1 < L.nd && t >= L.d[z].n_row_tiles * L.d[z].n_windows) {
        t -= L.d[z].n_row_tiles * L.d[z].n_windows;
        ++z;
    }
    // a private copy of the descriptor: a reference into the arguments at a
    // dynamic index had every stored row read its fields again; stack image
    // blockIdx.y reads and writes its own buffers
    PassDesc d = L.d[z];
    d.src = reinterpret_cast<const unsigned char*>(d.src) + (int64_t)blockIdx.y * d.src_step;
    d.dst = reinterpret_cast<unsigned char*>(d.dst) + (int64_t)blockIdx.y * d.dst_step;
    const int rt = t / d.n_windows;
    fwd_tile<TIn, T, GB, FIRST, LAST, OP, NW, SRCM>(d, rt, t - rt * d.n_windows, lds);
}

// Many passes (of many images) of one kind in one launch: block -> item ->
// group through the plan's item -> group map (one load), or without a map
// through a search of the groups' first_item prefix, as in the engine queue.
template <typename TIn, typename T, int GB, bool FIRST, bool LAST, int NW>
__global__ __launch_bounds__(NW * 64, 4) void fht_table_kernel(const EngineGroup* __restrict__ table, int n_groups,
                                                                int n_items, const int* __restrict__ group_of)
{
    __shared__ T lds[NW * 4 * kLdsRow];
    const int item = xcd_tile(blockIdx.x, n_items);
    if (item >= n_items) return;
    int lo = 0;
    if (group_of) {
        lo = group_of[item];
    } else {
        int hi = n_groups - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (table[mid].first_item <= item) lo = mid;
            else hi = mid - 1;
        }
    }
    // a private copy of the descriptor: read once, its fields stay in
    // registers (the table is global memory, which every store could alias)
    const PassDesc d = table[uniform(lo)].d;
    const int local = item - table[uniform(lo)].first_item;
    const int rt = local / d.n_windows;
    fwd_tile<TIn, T, GB, FIRST, LAST, 0, NW>(d, rt, local - rt * d.n_windows, lds);
}

// ------------------------------------------------- persistent forward engine
//
// One launch runs every tile of every pass of one depth G = 3 + GB (of every
// quadrant and image): an
// ordered queue of items, each one tile of one group.  Items are taken in
// queue order, so when a workgroup waits for the items of an earlier group,
// each of those items is already held by a running workgroup that never
// waits on a later item: the wait always ends.  A bounded spin turns a wait
// that does not end (a planner error) into an error flag instead of a hang.

__device__ __forceinline__ void wait_group(const unsigned* done, unsigned target, int limit, unsigned* err,
                                           int agent_acquire)
{
    int it = 0;
    while (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(4);
        if (++it > limit) {
            __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
    }
    // The producers wrote their band rows back to memory before counting
    // (release at agent scope).  An agent-scope acquire also invalidates this
    // XCD's caches; the lighter form relies on no cache of this launch holding
    // a line of the band before its group completed (bands are read only
    // after completion, and a launch starts with invalidated caches).
    if (agent_acquire) __atomic_thread_fence(__ATOMIC_ACQUIRE);
    else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <bool INLINE>
__device__ __forceinline__ const EngineGroup& engine_group(const EngineArgs& A, int g)
{
    if constexpr (INLINE) return A.g[g];
    else return A.table[g];
}

template <bool INLINE>
__device__ __forceinline__ int engine_find(const EngineArgs& A, int item)
{
    // last group whose first_item <= item
    int lo = 0, hi = A.n_groups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (engine_group<INLINE>(A, mid).first_item <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// INLINE: the groups travel in the kernel arguments (single images);
// otherwise they are read from a device table (batched plans).
template <typename TIn, typename T, int GB, bool INLINE>
__global__ __launch_bounds__(kThreads, 4) void fht_engine_kernel(const EngineArgs A)
{
    __shared__ T lds[kTileRows / 2 * kLdsRow];
    __shared__ int s_item;
    unsigned* head = A.sync;
    unsigned* err = A.sync + 1;
    unsigned* done = A.sync + 2;
    int seen_dep = -1;  // a dependency this workgroup has already seen complete
    if (threadIdx.x == 0) s_item = (int)atomicAdd(head, 1u);
    __syncthreads();
    int item = uniform(s_item);
    __syncthreads();
    for (;;) {
        if (item >= A.total_items) break;
        // take the next item now; its latency hides behind this tile
        unsigned next = 0;
        if (threadIdx.x == 0) next = atomicAdd(head, 1u);
        const int g = uniform(engine_find<INLINE>(A, item));
        const EngineGroup& E = engine_group<INLINE>(A, g);
        const int local = item - E.first_item;
        const int nw = E.d.n_windows;
        const int rt = local / nw;
        const int win = local - rt * nw;
        const int dep = E.dep;
        if (dep >= 0 && dep != seen_dep) {
            if (threadIdx.x == 0) wait_group(done + dep, (unsigned)E.dep_count, A.spin_limit, err, A.agent_acquire);
            __syncthreads();
            seen_dep = dep;
        }
        if (E.d.src_kind != SRC_BAND) {
            if (E.d.dst_kind == DST_HOUGH) fwd_tile<TIn, T, GB, true, true>(E.d, rt, win, lds);
            else fwd_tile<TIn, T, GB, true, false>(E.d, rt, win, lds);
        } else {
            if (E.d.dst_kind == DST_HOUGH) fwd_tile<TIn, T, GB, false, true>(E.d, rt, win, lds);
            else fwd_tile<TIn, T, GB, false, false>(E.d, rt, win, lds);
        }
        if (E.notify) {
            // every wave's stores complete, then one release makes them visible
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (threadIdx.x == 0) {
                __atomic_thread_fence(__ATOMIC_RELEASE);
                __hip_atomic_fetch_add(done + g, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (threadIdx.x == 0) s_item = (int)next;
        __syncthreads();
        item = uniform(s_item);
        __syncthreads();
    }
}

// ------------------------------------------------------ fused adjoint pass
//
// The transpose of one forward pass: the 2^G rows u*2^G + v of a block are
// read contiguously, the mini transform runs backwards (last GB stages
// transposed, then the LDS exchange with offsets moved to the write side, then
// the first 3 stages transposed) and row m is written with its column offset
// u*m added.  The halo sits at the low end of the tile.

// Hough gradient row (first adjoint pass): quadrant row s -> Hough row, x =
// +-xi, rolled columns.  Values arrive in memory order; the caller reverses
// mirrored rows after every row's loads are issued.
template <typename T>
__device__ __forceinline__ bool adj_issue_hough(const AdjDesc& d, int s_row, int xrow, int lane, T (&v)[8], int& e0)
{
    const int W = d.W;
    const bool skip = s_row == d.skip_row || s_row > d.row_limit;
    const T* src = reinterpret_cast<const T*>(d.src) + (long long)(d.row_base + d.row_sign * s_row) * d.src_ld;
    const int roll = d.shifted ? ((d.roll_a + d.roll_b * s_row) >> 1) : 0;
    e0 = lane_run_start(xrow, roll, lane, W, d.mirror);
    // the lane's 8 cells xi = xrow + 8*lane .. +7 inside the zero zone of row s
    bool black = false;
    if (d.black_ok) {
        const int x = mod_w(xrow, W) + 8 * lane;  // below W + 512: no second wrap needed
        const int xm = x >= W ? x - W : x;
        black = xm >= d.black_lo && xm + 8 <= d.black_lo + d.n - s_row;
    }
    const bool fast = !skip && !black && e0 + 8 <= W;
    load8<T>(fast ? src + e0 : zero_page<T>(), v);
    return !skip && !black && !fast;
}

template <typename T>
__device__ __forceinline__ void adj_patch_hough(const AdjDesc& d, int s_row, int e0, T (&v)[8])
{
    const T* src = reinterpret_cast<const T*>(d.src) + (long long)(d.row_base + d.row_sign * s_row) * d.src_ld;
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = src[run_col(e0, c, d.W, d.mirror)];
}

// Image-gradient stores.  Without accumulate the value is written; with it
// the value is added to the gradient already stored there (the earlier
// quadrants' sum s, giving s + value).
template <typename T, bool ACC>
__device__ __forceinline__ void acc_store8(T* p, const T (&v)[8])
{
    if constexpr (ACC) {
        T o[8];
        load8<T>(p, o);
#pragma unroll
        for (int c = 0; c < 8; ++c) o[c] = o[c] + v[c];
        store8<T>(p, o);
    } else {
        store8<T>(p, v);
    }
}

template <typename T, bool ACC>
__device__ __forceinline__ void acc_store1(T* p, T v)
{
    if constexpr (ACC) *p = *p + v;
    else *p = v;
}

template <typename T, int GB>
__device__ __forceinline__ void adj_exchange(T (&b)[8][8], T (&a)[8][8], T* lds, int wave, int lane)
{
    adj_stages_b<T, GB>(b);
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
                    lds_write8<T>(lds + (wa * 4 + (up & 3)) * kLdsRow + lane, uniform(up * rp), b[rho]);
                }
            }
            __syncthreads();
            {
                const T* lr = lds + wave * 4 * kLdsRow + lane;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                    for (int c = 0; c < 8; ++c) a[4 * h + rr][c] = lr[rr * kLdsRow + c * kPlane];
            }
            if (h == 0) __syncthreads();
        }
    }
}

// A private copy of descriptor k of a launch, for stack image im.
__device__ __forceinline__ AdjDesc adj_desc_for(const AdjLaunch& L, int k, int im)
{
    AdjDesc d = L.d[k];
    d.src = reinterpret_cast<const unsigned char*>(d.src) + (int64_t)im * d.src_step;
    d.dst = reinterpret_cast<unsigned char*>(d.dst) + (int64_t)im * d.dst_step;
    return d;
}

// One adjoint tile up to its stores: the forward pass's output rows of row
// tile rt at the window whose first own column is xi = x_lo (8 waves, wave
// 0..7 of them, exchange in lds), through the exchange and the stages, into
// a: lane l's register c is column xi = x_lo - 2^G + 8l + c of tile rows
// 8*wave .. 8*wave + 7.  Every wave reaches the exchange's barriers.
template <typename T, int GB, bool FIRST>
__device__ __forceinline__ void adj_compute(const AdjDesc& d, int rt, int x_lo, T* lds, int wave, int lane,
                                            T (&a)[8][8])
{
    constexpr int G = 3 + GB;
    constexpr int nmini_tile = 1 << (6 - G);
    const int j0 = d.j0;
    const int n_mini = d.n >> G;
    const int xw0 = x_lo - (1 << G);             // xi of the tile's column 0 (halo first)
    constexpr bool first = FIRST;                // reads the Hough gradient (else a band)
    const int W = d.W;

    // ---- load the forward pass's output rows (contiguous within a block)
    T b[8][8];
    {
        int e0[8];
        bool patch[8];
        bool any = false;
        const T* band = reinterpret_cast<const T*>(d.src);
#pragma unroll
        for (int rho = 0; rho < 8; ++rho) {
            const int rp = rho & ((1 << GB) - 1);
            const int q = rho >> GB;
            const int kappa = (wave << (3 - GB)) + q;
            const int t = kappa >> 3;
            const int up = kappa & 7;
            const int mu = rt * nmini_tile + t;
            patch[rho] = false;
            e0[rho] = 0;
            if (mu < n_mini) {
                const int B = mu >> j0;
                const int u = mu & ((1 << j0) - 1);
                const int s_row = (B << (j0 + G)) + (u << G) + (up << GB) + rp;
                if constexpr (first)
                    patch[rho] = adj_issue_hough<T>(d, s_row, xw0, lane, b[rho], e0[rho]);
                else
                    patch[rho] = issue_band_row<T>(band + (long long)s_row * d.src_ld, d.src_off, d.src_bw, W, xw0,
                                                   lane, b[rho], e0[rho]);
            } else {
                zero8(b[rho]);
            }
            any |= patch[rho];
        }
        if (first && d.mirror) {
#pragma unroll
            for (int rho = 0; rho < 8; ++rho) reverse8(b[rho]);
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
                    const int mu = rt * nmini_tile + t;
                    const int B = mu >> j0;
                    const int u = mu & ((1 << j0) - 1);
                    const int s_row = (B << (j0 + G)) + (u << G) + (up << GB) + rp;
                    if constexpr (first) adj_patch_hough<T>(d, s_row, e0[rho], b[rho]);
                    else patch_band_row<T>(band + (long long)s_row * d.src_ld, d.src_bw, W, e0[rho], b[rho]);
                }
            }
        }
    }

    adj_exchange<T, GB>(b, a, lds, wave, lane);
    adj_stage<T, 2>(a);
    adj_stage<T, 1>(a);
    adj_stage<T, 0>(a);
}

// ACC: the image pass that adds its values to the stored gradient (the
// descriptors' accumulate flag); a separate instantiation keeps that code
// out of every other adjoint kernel.
template <typename T, int GB, bool FIRST, bool LAST, bool ACC = false>
__device__ __forceinline__ void adj_tile(const AdjDesc& d, int rt, int win, T* lds)
{
    constexpr int G = 3 + GB;
    constexpr int VW = kWinCols - (1 << G);
    constexpr int nmini_tile = 1 << (6 - G);
    const int lane = threadIdx.x & 63;
    const int wave = uniform(threadIdx.x >> 6);
    const int j0 = d.j0;
    const int n_mini = d.n >> G;
    const int x_lo = d.x_start + win * VW;
    const int xw0 = x_lo - (1 << G);
    const int W = d.W;
    T a[8][8];
    adj_compute<T, GB, FIRST>(d, rt, x_lo, lds, wave, lane, a);

    // ---- store row m of each mini transform at its offset u*m
    const int wc0 = 8 * lane;
    if (wc0 < (1 << G)) return;
    const int xi = xw0 + wc0;  // xi of register 0 before the offset
    const int tr0 = wave * 8;
    const int t = tr0 >> G;
    const int mu = rt * nmini_tile + t;
    if (mu >= n_mini) return;
    const int B = mu >> j0;
    const int u = mu & ((1 << j0) - 1);
    if constexpr (!LAST) {
        // band: window columns [0, W) are covered once; column z of row m lands
        // on z + u*m, a bijection of the cyclic row
        if (xi >= W) return;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int m = (tr0 + r) & ((1 << G) - 1);
            const int R = (B << (j0 + G)) + (m << j0) + u;
            T* dst = reinterpret_cast<T*>(d.dst) + (long long)R * d.dst_ld;
            const int e0 = wrap_up(mod_w(xw0 + u * m + d.dst_off, W) + wc0, W);
            if (xi + 8 <= W && e0 + 8 <= d.dst_bw) {
                store8<T>(dst + e0, a[r]);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (xi + c < W) {
                        int e = e0 + c;
                        if (e >= W) e -= W;
                        if (e < d.dst_bw) dst[e] = a[r][c];
                    }
                }
            }
        }
        return;
    }
    // image (the first forward pass has u = 0: no offset remains); x = +-xi.
    // The windows cover xi in [x_start, x_start + cols) once, which maps onto
    // image columns 0..cols-1; anything past that is another window's.
    const int cols = d.dst_kind == 1 ? d.img_w : d.img_h;
    const int rel = xi - d.x_start;
    if (rel >= cols) return;
    const int e0 = d.mirror ? wrap_down(mod_w(-xi - 7, W), W) : wrap_up(mod_w(xi, W), W);
    const bool full_run = rel + 8 <= cols && e0 + 8 <= cols;
    if (d.dst_kind == 1) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int R = (B << G) + ((tr0 + r) & ((1 << G) - 1));
            if (R >= d.img_h) continue;
            T* p = reinterpret_cast<T*>(d.dst) + (long long)R * d.dst_ld;
            if (full_run) {
                T v[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) v[c] = d.mirror ? a[r][7 - c] : a[r][c];
                acc_store8<T, ACC>(p + e0, v);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int e = run_col(e0, c, W, d.mirror);
                    if (rel + c < cols && e < cols) acc_store1<T, ACC>(p + e, a[r][c]);
                }
            }
        }
    } else {
        // transposed image: rows R0..R0+7 are image columns, contiguous in memory
        const int R0 = (B << G) + (tr0 & ((1 << G) - 1));
        const bool all_cols = R0 + 8 <= d.img_w;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int e = run_col(e0, c, W, d.mirror);  // image row
            if (rel + c >= cols || e >= d.img_h) continue;
            T* p = reinterpret_cast<T*>(d.dst) + (long long)e * d.dst_ld + R0;
            T v[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) v[r] = a[r][c];
            if (all_cols) {
                acc_store8<T, ACC>(p, v);
            } else {
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (R0 + r < d.img_w) acc_store1<T, ACC>(p + r, v[r]);
            }
        }
    }
}

template <typename T, int GB, bool FIRST, bool LAST, bool ACC>
__global__ __launch_bounds__(kThreads, 4) void fht_adj_pass_kernel(const AdjLaunch L)
{
    __shared__ T lds[kTileRows / 2 * kLdsRow];
    // a private copy: its fields stay in registers across the stores
    const int k = uniform((int)blockIdx.z % L.nd);
    const AdjDesc d = adj_desc_for(L, k, uniform((int)blockIdx.z / L.nd));
    if ((int)blockIdx.x >= d.n_windows || (int)blockIdx.y >= d.n_row_tiles) return;
    adj_tile<T, GB, FIRST, LAST, ACC>(d, blockIdx.y, blockIdx.x, lds);
}

// Image pass of a mirror pair of quadrants (1 and 2, or 3 and 4) over the
// same image region, one 16-wave workgroup per tile.  Descriptor 2z is the
// unmirrored quadrant U (waves 0-7), 2z + 1 the mirrored one M (waves 8-15);
// both have the same n, stage split, row tiles and image columns.  U's
// window w covers image columns [c0, c0 + VW), c0 = w * VW, at xi = x; M
// covers the same columns at xi = W - x, from its own first column
// xi = W - c0 - VW + 1.  After the stages M's values go through LDS (the two
// exchange regions, free again) to the U lane holding the same image cell,
// and U's waves store M + U, or with ACC (s + M) + U where s is the
// gradient already stored there (the earlier quadrants' sum, in quadrant
// order).  Both halves run the same loads, exchange barriers and stages.
template <typename T, int GB, bool FIRST, bool ACC>
__global__ __launch_bounds__(2 * kThreads, 4) void fht_adj_pair_kernel(const AdjLaunch L)
{
    __shared__ T lds[kTileRows * kLdsRow];
    constexpr int G = 3 + GB;
    constexpr int VW = kWinCols - (1 << G);
    constexpr int nmini_tile = 1 << (6 - G);
    constexpr int kCbRow = kWinCols;  // combine buffer: one row per tile row
    static_assert(kTileRows * kCbRow <= kTileRows * kLdsRow, "combine buffer exceeds the exchange regions");
    // pair p of stack image im: z = im * (nd / 2) + p; the whole workgroup
    // leaves together (U's counts bound the pair)
    const int np = L.nd >> 1;
    const int pz = uniform((int)blockIdx.z % np);
    if ((int)blockIdx.x >= L.d[2 * pz].n_windows || (int)blockIdx.y >= L.d[2 * pz].n_row_tiles) return;
    const int half = uniform((int)threadIdx.x >> 9);
    const int wave = uniform(((int)threadIdx.x >> 6) & 7);
    const int lane = threadIdx.x & 63;
    const AdjDesc d = adj_desc_for(L, 2 * pz + half, uniform((int)blockIdx.z / np));
    const int c0 = blockIdx.x * VW;
    const int x_lo = half == 0 ? c0 : d.W - c0 - VW + 1;
    T a[8][8];
    adj_compute<T, GB, FIRST>(d, blockIdx.y, x_lo, lds + half * (kTileRows / 2 * kLdsRow), wave, lane, a);
    __syncthreads();  // every wave is done with both exchange regions

    // image column of register c: U lane l, c0 - 2^G + 8l + c; M lane l,
    // c0 + 511 - 8l - c.  Offsets o = column - c0 in [0, VW) are the lanes
    // with 8l >= 2^G (the others hold the halo).
    const bool own = 8 * lane >= (1 << G);
    T* cb = lds + wave * 8 * kCbRow;
    if (half == 1 && own) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            T* q = cb + r * kCbRow + (kWinCols - 8) - 8 * lane;  // offsets 504 - 8l .. 511 - 8l
#pragma unroll
            for (int c = 0; c < 8; ++c) q[c] = a[r][7 - c];
        }
    }
    __syncthreads();
    if (half == 1 || !own) return;

    // ---- stores (the image pass: j0 = 0, row m of mini transform mu is
    // tile row (mu << G) + m).  M's values are read from LDS next to their
    // use, a row (or column) at a time, so that only U's tile stays in
    // registers.
    const T* mrow = cb + 8 * lane - (1 << G);  // M's value at U's register (r, c): mrow[r * kCbRow + c]
    const int xi = c0 - (1 << G) + 8 * lane;   // image column of register 0
    const int tr0 = wave * 8;
    const int mu = blockIdx.y * nmini_tile + (tr0 >> G);
    if (mu >= (d.n >> G)) return;
    const int cols = d.dst_kind == 1 ? d.img_w : d.img_h;
    if (xi >= cols) return;
    const bool full_run = xi + 8 <= cols;
    if (d.dst_kind == 1) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int R = (mu << G) + ((tr0 + r) & ((1 << G) - 1));
            if (R >= d.img_h) continue;
            T mv[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) mv[c] = mrow[r * kCbRow + c];
            T* p = reinterpret_cast<T*>(d.dst) + (long long)R * d.dst_ld + xi;
            if (full_run) {
                T v[8];
                if constexpr (ACC) {
                    load8<T>(p, v);
#pragma unroll
                    for (int c = 0; c < 8; ++c) v[c] = (v[c] + mv[c]) + a[r][c];
                } else {
#pragma unroll
                    for (int c = 0; c < 8; ++c) v[c] = mv[c] + a[r][c];
                }
                store8<T>(p, v);
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (xi + c < cols) p[c] = ACC ? (p[c] + mv[c]) + a[r][c] : mv[c] + a[r][c];
            }
        }
    } else {
        // transposed image: tile rows R0..R0+7 are image columns, register c
        // is image row xi + c
        const int R0 = (mu << G) + (tr0 & ((1 << G) - 1));
        const bool all_cols = R0 + 8 <= d.img_w;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (xi + c >= cols) continue;
            T mv[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) mv[r] = mrow[r * kCbRow + c];
            T* p = reinterpret_cast<T*>(d.dst) + (long long)(xi + c) * d.dst_ld + R0;
            if (all_cols) {
                T v[8];
                if constexpr (ACC) {
                    load8<T>(p, v);
#pragma unroll
                    for (int r = 0; r < 8; ++r) v[r] = (v[r] + mv[r]) + a[r][c];
                } else {
#pragma unroll
                    for (int r = 0; r < 8; ++r) v[r] = mv[r] + a[r][c];
                }
                store8<T>(p, v);
            } else {
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (R0 + r < d.img_w) p[r] = ACC ? (p[r] + mv[r]) + a[r][c] : mv[r] + a[r][c];
            }
        }
    }
}

// -------------------------------------------- direct form for n <= 4 rows

template <typename TIn, typename T>
__device__ __forceinline__ T src_value(const PassDesc& d, int R, int x)
{
    const int W = d.W;
    const int e = mod_pos((long long)x - shear_of_row(R, d.S1, d.n), W);
    const int es = d.scale_num ? (int)(((long long)e * d.scale_den) / d.scale_num) : e;
    const TIn* img = reinterpret_cast<const TIn*>(d.src);
    if (d.src_kind == SRC_IMAGE)
        return (R < d.img_h && e < d.img_w) ? to_acc<T>(img[(long long)R * d.src_ld + es]) : (T)0;
    return (R < d.img_w && e < d.img_h) ? to_acc<T>(img[(long long)es * d.src_ld + R]) : (T)0;
}

// The same add tree as K stages of the recurrence, evaluated top-down in x
// (direction -1 for mirrored quadrants).
template <typename TIn, typename T, int K, int OP>
__device__ T direct_sum(const PassDesc& d, int base, int s, int x)
{
    if constexpr (K == 0) {
        return src_value<TIn, T>(d, base, x);
    } else {
        const int sub = s >> 1;
        const int dir = d.mirror ? -1 : 1;
        const T top = direct_sum<TIn, T, K - 1, OP>(d, base, sub, x);
        const T bot = direct_sum<TIn, T, K - 1, OP>(d, base + (1 << (K - 1)), sub,
                                                   mod_pos((long long)x + dir * (s - sub), d.W));
        return combine<OP>(top, bot);
    }
}

template <typename TIn, typename T, int K, int OP>
__global__ __launch_bounds__(256) void fht_direct_kernel(const PassLaunch L)
{
    // z = stack image * nd + descriptor
    PassDesc d = L.d[(int)blockIdx.z % L.nd];
    const int64_t im = (int)blockIdx.z / L.nd;
    d.src = reinterpret_cast<const unsigned char*>(d.src) + im * d.src_step;
    d.dst = reinterpret_cast<unsigned char*>(d.dst) + im * d.dst_step;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (x >= d.W || s >= d.n || s > d.row_limit || s == d.skip_row) return;
    const T v = direct_sum<TIn, T, K, OP>(d, 0, s, x);
    T* dst = reinterpret_cast<T*>(d.dst) + (long long)(d.row_base + d.row_sign * s) * d.dst_ld;
    const int roll = d.shifted ? ((d.roll_a + d.roll_b * s) >> 1) : 0;
    dst[mod_pos((long long)x + roll, d.W)] = v;
}

// Direct quadrants (n <= 4 rows) of many images in one launch: one thread
// per Hough cell, cells of consecutive groups back to back (first_item
// prefix, n x W cells per group).
template <typename TIn, typename T>
__global__ __launch_bounds__(256) void fht_table_direct_kernel(const EngineGroup* __restrict__ table, int n_groups,
                                                                int n_items)
{
    const int item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= n_items) return;
    int lo = 0, hi = n_groups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].first_item <= item) lo = mid;
        else hi = mid - 1;
    }
    const PassDesc& d = table[lo].d;
    const int local = item - table[lo].first_item;
    const int s = local / d.W;
    const int x = local - s * d.W;
    if (s >= d.n || s > d.row_limit || s == d.skip_row) return;
    T v;
    if (d.n == 1) v = direct_sum<TIn, T, 0, 0>(d, 0, s, x);
    else if (d.n == 2) v = direct_sum<TIn, T, 1, 0>(d, 0, s, x);
    else v = direct_sum<TIn, T, 2, 0>(d, 0, s, x);
    T* dst = reinterpret_cast<T*>(d.dst) + (long long)(d.row_base + d.row_sign * s) * d.dst_ld;
    const int roll = d.shifted ? ((d.roll_a + d.roll_b * s) >> 1) : 0;
    dst[mod_pos((long long)x + roll, d.W)] = v;
}

// Adjoint for n <= 4 rows: B_j from B_{j+1} by the transposed stage, top-down
// in x.
template <typename T, int J, int K>
__device__ T adj_direct(const AdjDesc& d, int row, int x)
{
    if constexpr (J == K) {
        if (row == d.skip_row || row > d.row_limit) return (T)0;
        const T* src = reinterpret_cast<const T*>(d.src) + (long long)(d.row_base + d.row_sign * row) * d.src_ld;
        const int roll = d.shifted ? ((d.roll_a + d.roll_b * row) >> 1) : 0;
        return src[mod_pos((long long)x + roll, d.W)];
    } else {
        const int blk = 1 << J;
        const int base = (row / (2 * blk)) * (2 * blk);
        const int i = row - base;
        if (i < blk) {
            return adj_direct<T, J + 1, K>(d, base + 2 * i, x) + adj_direct<T, J + 1, K>(d, base + 2 * i + 1, x);
        }
        const int u = i - blk;
        const int dir = d.mirror ? -1 : 1;
        return adj_direct<T, J + 1, K>(d, base + 2 * u, mod_pos((long long)x - dir * u, d.W)) +
               adj_direct<T, J + 1, K>(d, base + 2 * u + 1, mod_pos((long long)x - dir * (u + 1), d.W));
    }
}

template <typename T, int K>
__global__ __launch_bounds__(256) void fht_adj_direct_kernel(const AdjLaunch L)
{
    const AdjDesc d = adj_desc_for(L, (int)blockIdx.z % L.nd, (int)blockIdx.z / L.nd);
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int R = blockIdx.y;
    if (R >= d.n) return;
    // dst_kind 1: image, 2: transposed image, 0: the full n x W source buffer
    const int cols = d.dst_kind == 1 ? d.img_w : (d.dst_kind == 2 ? d.img_h : d.W);
    const int rows = d.dst_kind == 1 ? d.img_h : (d.dst_kind == 2 ? d.img_w : d.n);
    if (x >= cols || R >= rows) return;
    const T v = adj_direct<T, 0, K>(d, R, x);
    T* p = d.dst_kind == 2 ? reinterpret_cast<T*>(d.dst) + (long long)x * d.dst_ld + R
                           : reinterpret_cast<T*>(d.dst) + (long long)R * d.dst_ld + x;
    *p = d.accumulate ? *p + v : v;
}

// ------------------------------------------------ angle-range adjoint tail

// The gradient of the sheared padded source, a0[r, xi] (n x W), read back
// as the gradient of the source cell (r, c), xi = c + sigma(r) (section 4),
// cropped to the image.  One thread per image cell, consecutive x.
template <typename T>
__global__ __launch_bounds__(256) void fht_unshear_kernel(const T* a0, int W, int n, int S1, T* img, int64_t ld_img,
                                                          int w, int h, int transposed)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= w) return;
    for (int y = blockIdx.y; y < h; y += gridDim.y) {  // grid y capped at 65535
        const int r = transposed ? x : y;
        const int c = transposed ? y : x;
        const int xi = mod_pos((long long)c + shear_of_row(r, S1, n), W);
        img[(long long)y * ld_img + x] = a0[(long long)r * W + xi];
    }
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
    static_assert(sizeof(T) == 4, "4-byte cells");
    typedef unsigned u32x4u __attribute__((ext_vector_type(4), aligned(4)));
    const int W = hp + wp;
    const int rows = 2 * (hp + wp) - 3;
    // four consecutive output cells per thread
    const int x0 = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
    if (x0 >= W) return;
    // grid y is capped (65535); rows beyond it are taken in strides
    for (int r = blockIdx.y; r < rows; r += gridDim.y) {
        int roll = row_roll(r, hp, wp) % W;
        if (inverse) roll = (W - roll) % W;
        int src = x0 - roll;
        if (src < 0) src += W;
        const T* pin = in + (long long)r * ld_in;
        T* po = out + (long long)r * ld_out + x0;
        if (x0 + 4 <= W && src + 4 <= W) {
            // the four source cells are consecutive: one 16-byte load and
            // store (dword alignment suffices on gfx950)
            *reinterpret_cast<u32x4u*>(po) = *reinterpret_cast<const u32x4u*>(pin + src);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (x0 + c >= W) break;
                int s = src + c;
                if (s >= W) s -= W;
                po[c] = pin[s];
            }
        }
    }
}

}  // namespace fht
