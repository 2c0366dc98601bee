// Internal declarations shared by the C ABI (fht_api.hip) and the kernels
// (fht_kernels.hip).  Not installed; the public interface is include/fht.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fht {

// Tile geometry of the fused pass kernel.  One workgroup holds 64 rows x 512
// columns: 8 waves, each lane owns 8 consecutive columns of 8 rows.
constexpr int kTileRows = 64;
constexpr int kLaneCols = 8;
constexpr int kWinCols = 512;           // columns loaded per tile
constexpr int kThreads = 512;
constexpr int kPlane = 72;              // LDS: 8 planes of 72 words per row (column-swizzled)
constexpr int kLdsRow = 8 * kPlane;     // 576 words per tile row
constexpr int kLdsOffNeg = 56;          // LDS column bias for the negative direction
constexpr int kMaxG = 6;                // stages per pass (3 in registers + up to 3 after the exchange)

enum SrcKind : int { SRC_IMAGE = 0, SRC_IMAGE_T = 1, SRC_BAND = 2 };
enum DstKind : int { DST_BAND = 0, DST_HOUGH = 1 };

// One pass (G consecutive stages) over one quadrant.
struct PassDesc {
    const void* src;      // image (first pass) or band of the previous pass
    void* dst;            // band of this pass or the Hough image
    int64_t src_ld;       // elements
    int64_t dst_ld;       // elements
    int src_kind;         // SrcKind
    int dst_kind;         // DstKind
    int img_w, img_h;     // image extent (image sources)
    int n;                // rows of the quadrant (h' or w')
    int W;                // columns (w' + h')
    int j0;               // stages completed before this pass
    int dir;              // +1 (quadrants 1, 4) or -1 (quadrants 2, 3)
    int src_off, src_bw;  // band source: index = (x + src_off) mod W, nonzero iff index < src_bw
    int dst_off, dst_bw;  // band destination, same convention
    int S1;               // first-pass shear (angle range); 0 = none
    int x_start;          // logical column of the first output column of window 0
    int n_windows;        // windows of (512 - 2^G) output columns
    int n_row_tiles;      // ceil(n / 64)
    int row_limit;        // output rows (local shift within a 2^(j0+G) block) above it are not needed
    int row_base;         // Hough destination: row = row_base + row_sign * s
    int row_sign;
    int skip_row;         // shift whose row is not written (-1: none)
    int shifted;          // apply the fhtshift roll (roll_a + roll_b * s) >> 1
    int roll_a, roll_b;
};

constexpr int kMaxDescs = 4;
struct PassLaunch {
    PassDesc d[kMaxDescs];
    int nd;
};

// Adjoint pass: the transpose of one forward pass.
struct AdjDesc {
    const void* src;      // Hough gradient (first adjoint pass) or band
    void* dst;            // band or the image gradient (accumulated over quadrants)
    int64_t src_ld, dst_ld;
    int src_kind;         // 0: Hough rows, 1: band
    int dst_kind;         // 0: band, 1: image, 2: image transposed
    int accumulate;       // image destinations: add to the existing value
    int img_w, img_h;
    int n, W, j0, dir;
    int src_off, src_bw;
    int dst_off, dst_bw;
    int x_start, n_windows, n_row_tiles;
    int row_base, row_sign, skip_row;  // Hough source row mapping
    int shifted, roll_a, roll_b;
};
struct AdjLaunch {
    AdjDesc d[kMaxDescs];
    int nd;
};

hipError_t launch_pass(const PassLaunch& L, int G, bool first, bool last, int in_t, int acc_t, hipStream_t s);
hipError_t launch_direct(const PassLaunch& L, int k, int in_t, int acc_t, hipStream_t s);
hipError_t launch_adjoint_pass(const AdjLaunch& L, int G, bool first, bool last, int t, hipStream_t s);
hipError_t launch_adjoint_direct(const AdjLaunch& L, int k, int t, hipStream_t s);
hipError_t launch_zero(void* p, int64_t rows, int64_t cols, int64_t ld, int elem_bytes, hipStream_t s);
hipError_t launch_shift(const void* in, int64_t ld_in, void* out, int64_t ld_out, int elem_bytes,
                        int hp, int wp, int inverse, hipStream_t s);

}  // namespace fht
