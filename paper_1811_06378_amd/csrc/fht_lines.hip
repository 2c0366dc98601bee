// From Hough cells back to the image: the segment a cell's pattern covers
// (sections 3.2 and 3.3), and local maxima of a Hough image on the GPU.
#include "fht.h"
#include "fht_internal.h"
#include "fht_plan.h"

namespace fht {

// D_n(s, y): column offset of row y of the dyadic pattern with shift s over
// n = 2^k rows; bit k-1-j of y contributes (s >> j) - (s >> (j+1)).
static int64_t pattern_offset(int64_t n, int64_t s, int64_t y)
{
    int k = 0;
    while ((int64_t(1) << k) < n) ++k;
    int64_t d = 0;
    for (int j = 0; j < k; ++j)
        if ((y >> (k - 1 - j)) & 1) d += (s >> j) - (s >> (j + 1));
    return d;
}

static int64_t mod64(int64_t a, int64_t m)
{
    a %= m;
    return a < 0 ? a + m : a;
}

// Strict local maximum over a (2r+1)^2 neighbourhood, cyclic in columns (the
// Hough image is cyclic in x0), clipped in rows; equal values are ordered by
// their linear index, so a plateau yields one peak.
template <typename T>
__global__ __launch_bounds__(256) void fht_peaks_kernel(const T* H, int64_t rows, int64_t cols, int64_t ld,
                                                        int radius, double threshold, int64_t* out, int max_out,
                                                        unsigned* count)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {  // grid y capped at 65535
        const T v = H[r * ld + c];
        if (!((double)v > threshold)) continue;
        const int64_t me = r * cols + c;
        bool peak = true;
        for (int dr = -radius; dr <= radius && peak; ++dr) {
            const int64_t rr = r + dr;
            if (rr < 0 || rr >= rows) continue;
            for (int dc = -radius; dc <= radius; ++dc) {
                if (dr == 0 && dc == 0) continue;
                int64_t cc = c + dc;
                if (cc < 0) cc += cols;
                if (cc >= cols) cc -= cols;
                const T u = H[rr * ld + cc];
                if (u > v || (u == v && rr * cols + cc < me)) {
                    peak = false;
                    break;
                }
            }
        }
        if (!peak) continue;
        const unsigned slot = atomicAdd(count, 1u);
        if ((int)slot < max_out) out[slot] = me;
    }
}

__global__ void fht_zero_u32_kernel(unsigned* p) { *p = 0u; }

}  // namespace fht

using namespace fht;

extern "C" {

int fht_cell_segment(int w, int h, unsigned quads, int64_t row, int64_t x0, int shifted, int32_t* seg)
{
    int rc = check_sides(w, h);
    if (rc) return rc;
    if (!seg) return fail(FHT_ERR_INVALID, "null segment output");
    const int64_t hp = pow2_ceil(h), wp = pow2_ceil(w), W = hp + wp;
    int q = 0;
    int64_t s = 0;
    if (quads == FHT_FULL) {
        const int64_t rows = 2 * (hp + wp) - 3;
        if (row < 0 || row >= rows) return fail(FHT_ERR_INVALID, "row %lld outside 0..%lld", (long long)row,
                                                (long long)(rows - 1));
        // the quadrant order of section 3.3 with its shared rows
        if (row < hp) { q = 1; s = hp - 1 - row; }
        else if (row <= 2 * hp - 2) { q = 2; s = row - hp + 1; }
        else if (row <= 2 * hp + wp - 3) { q = 3; s = 2 * hp + wp - 3 - row; }
        else { q = 4; s = row - (2 * hp + wp - 3); }
    } else {
        if (quads != FHT_Q1 && quads != FHT_Q2 && quads != FHT_Q3 && quads != FHT_Q4)
            return fail(FHT_ERR_INVALID, "quads must be FHT_FULL or one quadrant");
        if (shifted) return fail(FHT_ERR_INVALID, "fhtshift applies to the full Hough image only");
        q = quads == FHT_Q1 ? 1 : quads == FHT_Q2 ? 2 : quads == FHT_Q3 ? 3 : 4;
        const int64_t n = q <= 2 ? hp : wp;
        if (row < 0 || row >= n) return fail(FHT_ERR_INVALID, "row %lld outside 0..%lld", (long long)row,
                                             (long long)(n - 1));
        s = row;
    }
    if (x0 < 0 || x0 >= W) return fail(FHT_ERR_INVALID, "x0 %lld outside 0..%lld", (long long)x0, (long long)(W - 1));
    const int64_t n = q <= 2 ? hp : wp;
    if (shifted) {
        // fhtshift rolled the row right by floor((n +- s) / 2) (section 5)
        const int64_t roll = (q == 1 || q == 4) ? (n + s) / 2 : (n - s) / 2;
        x0 = mod64(x0 - roll, W);
    }
    const int dir = (q == 1 || q == 4) ? 1 : -1;
    const bool transposed = q >= 3;
    int64_t first = -1, last = -1, count = 0;
    int64_t xa = 0, ya = 0, xb = 0, yb = 0;
    for (int64_t y = 0; y < n; ++y) {
        const int64_t x = mod64(x0 + dir * pattern_offset(n, s, y), W);  // cases a and b: cyclic columns
        const int64_t X = transposed ? y : x, Y = transposed ? x : y;
        if (X >= w || Y >= h) continue;  // padding: outside the image
        if (first < 0) { first = y; xa = X; ya = Y; }
        last = y;
        xb = X;
        yb = Y;
        ++count;
    }
    // case c: the pattern lies in the extension only (black zone), no segment
    seg[0] = (int32_t)xa; seg[1] = (int32_t)ya; seg[2] = (int32_t)xb; seg[3] = (int32_t)yb;
    seg[4] = (int32_t)count;
    (void)last;
    return FHT_OK;
}

int fht_peaks(const void* hough, int t, int64_t rows, int64_t cols, int64_t ld, int radius, double threshold,
              int64_t* out, int max_out, unsigned* count, void* stream)
{
    if (!hough || !out || !count) return fail(FHT_ERR_INVALID, "null pointer");
    if (t != FHT_I32 && t != FHT_F32) return fail(FHT_ERR_INVALID, "Hough type must be I32 or F32");
    if (rows < 1 || cols < 1 || ld < cols) return fail(FHT_ERR_INVALID, "bad Hough shape");
    if (radius < 1 || radius > 64 || 2 * radius + 1 > cols) return fail(FHT_ERR_INVALID, "radius %d", radius);
    if (max_out < 1) return fail(FHT_ERR_INVALID, "max_out %d", max_out);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(fht_zero_u32_kernel, dim3(1), dim3(1), 0, s, count);
    const dim3 grid((unsigned)((cols + 255) / 256), (unsigned)(rows < 65535 ? rows : 65535));
    if (t == FHT_I32)
        hipLaunchKernelGGL(fht_peaks_kernel<int>, grid, dim3(256), 0, s, (const int*)hough, rows, cols, ld, radius,
                           threshold, out, max_out, count);
    else
        hipLaunchKernelGGL(fht_peaks_kernel<float>, grid, dim3(256), 0, s, (const float*)hough, rows, cols, ld,
                           radius, threshold, out, max_out, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "peaks launch");
    return FHT_OK;
}

}  // extern "C"
