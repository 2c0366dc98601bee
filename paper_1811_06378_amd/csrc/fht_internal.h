// Internal declarations shared by the C ABI (fht_api.hip, fht_batch.hip) and
// the kernels (fht_device.h, instantiated in fht_fwd_*.hip / fht_adj_*.hip).
// Not installed; the public interface is include/fht.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace fht {

// Tile geometry of the fused pass kernel.  One workgroup holds 64 rows x 512
// columns: 8 waves, each lane owns 8 consecutive columns of 8 rows.
constexpr int kTileRows = 64;
constexpr int kNarrowRows = 32;         // narrow tiles: 4 waves, passes of at most 5 stages
constexpr int kLaneCols = 8;
constexpr int kWinCols = 512;           // columns loaded per tile
constexpr int kThreads = 512;
constexpr int kPlane = 72;              // LDS: 8 planes of 72 words per row (column-swizzled)
constexpr int kLdsRow = 8 * kPlane;     // 576 words per tile row
constexpr int kMaxG = 6;                // stages per pass (3 in registers + up to 3 after the exchange)

enum SrcKind : int { SRC_IMAGE = 0, SRC_IMAGE_T = 1, SRC_BAND = 2 };
enum DstKind : int { DST_BAND = 0, DST_HOUGH = 1 };

// One pass (G consecutive stages) over one quadrant.
//
// Columns are handled in the quadrant's own coordinate xi = dir * x (mod W):
// in xi every stage reads its second row shifted towards larger xi, so one
// kernel serves all four quadrants.  Only the image loads of the first pass
// and the Hough stores of the last pass map xi back to x (mirror = dir < 0).
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
    int G;                // stages in this pass (3..6)
    int mirror;           // 1 for quadrants 2, 3 (x = -xi)
    int src_off, src_bw;  // band source: index = (xi + src_off) mod W, nonzero iff index < src_bw
    int dst_off, dst_bw;  // band destination, same convention
    int S1;               // first-pass shear (angle range, unmirrored quadrants); 0 = none
    int x_start;          // xi of the first stored column of window 0
    int n_windows;        // windows of (512 - 2^G) stored columns
    int n_row_tiles;      // ceil(n / 64)
    int row_limit;        // rows (local shift within a 2^(j0+G) block) above it are not needed
    int row_base;         // Hough destination: row = row_base + row_sign * s
    int row_sign;
    int skip_row;         // shift whose row is not written (-1: none)
    int shifted;          // apply the fhtshift roll (roll_a + roll_b * s) >> 1
    int roll_a, roll_b;
    int black_lo;         // last pass: xi in [black_lo, black_lo + n - s) is structurally zero in row s
    int black_ok;         // 1: tiles wholly inside that zone are written as zeros without loads
    int scale_num, scale_den;  // first pass: source sample floor(x * den / num) along the
                               // sheared axis (section 4 scale); 0 = no scaling
    int tile_rows;        // 64 (8 waves) or 32 (4 waves, G <= 5); n_row_tiles = ceil(n / tile_rows)
    int64_t src_step;     // bytes from one stack image's source to the next's (pass launches)
    int64_t dst_step;     // bytes from one stack image's destination to the next's
};

// Up to 4 quadrants' descriptors of one pass kind, for n_img images of a
// stack: image i (grid y; z for the direct kernel) has every descriptor's
// src and dst advanced by i * src_step and i * dst_step.
constexpr int kMaxDescs = 4;
struct PassLaunch {
    PassDesc d[kMaxDescs];
    int nd;
    int n_tiles;  // sum of n_row_tiles * n_windows (filled by the launcher)
    int n_img;    // < 1 counts as 1
};

// Adjoint pass: the transpose of one forward pass, in the same xi coordinate.
struct AdjDesc {
    const void* src;      // Hough gradient (first adjoint pass) or band
    void* dst;            // band or the image gradient (accumulated over quadrants)
    int64_t src_ld, dst_ld;
    int src_kind;         // 0: Hough rows, 1: band
    int dst_kind;         // 0: band, 1: image, 2: image transposed
    int accumulate;       // image destination: 1 = add the value to the one stored there
                          //   (the earlier quadrants' sum), 0 = store it
    int img_w, img_h;
    int n, W, j0, G, mirror;
    int src_off, src_bw;
    int dst_off, dst_bw;
    int x_start, n_windows, n_row_tiles;
    int row_base, row_sign, skip_row;  // Hough source row mapping
    int row_limit;        // Hough rows (shifts) above it read as zero (angle range: S)
    int shifted, roll_a, roll_b;
    int black_lo;         // Hough source: xi in [black_lo, black_lo + n - s) of row s is
    int black_ok;         // the structurally zero zone; 1: read it as zero (no shear)
    int64_t src_step;     // bytes from one stack image's source to the next's
    int64_t dst_step;     // bytes from one stack image's destination to the next's
};
// Up to 4 quadrants' descriptors of one adjoint pass kind, for n_img images
// of a stack: launch z = image * nd + descriptor, and image i's descriptors
// have src and dst advanced by i * src_step and i * dst_step.
constexpr int kMaxAdjDescs = 4;
struct AdjLaunch {
    AdjDesc d[kMaxAdjDescs];
    int nd;
    int n_img;  // < 1 counts as 1
};

// Persistent forward engine: an ordered queue of items (one tile each) drawn
// from groups (one pass of one quadrant of one image).  A group may wait for
// every item of one earlier group (its previous pass).
struct EngineGroup {
    PassDesc d;
    int first_item;       // queue index of the group's first item
    int count;            // items = n_row_tiles * n_windows
    int dep;              // group whose items must all be done first (-1: none)
    int dep_count;        // item count of that group
    int notify;           // 1: count this group's finished items
    int pad_;
};

constexpr int kEngineInline = 12;
struct EngineArgs {
    EngineGroup g[kEngineInline];  // used when table == nullptr
    const EngineGroup* table;      // device table (batched plans)
    int n_groups;
    int total_items;
    unsigned* sync;                // [0] queue head, [1] error flag, [2 + g] items done in group g
    int spin_limit;                // bounded dependency wait (iterations)
    int agent_acquire;             // 1: agent-scope acquire after a wait (invalidates the XCD's caches)
};

inline size_t engine_sync_bytes(int n_groups) { return ((size_t)(n_groups + 2) * 4 + 255) / 256 * 256; }

// op: 0 = sum along the patterns, 1 = max
hipError_t launch_pass(const PassLaunch& L, int in_t, int acc_t, hipStream_t s, int op = 0);
hipError_t launch_direct(const PassLaunch& L, int k, int in_t, int acc_t, hipStream_t s, int op = 0);
hipError_t launch_engine(const EngineArgs& A, int G, int grid, int in_t, int acc_t, hipStream_t s);
// table: device array of n_groups groups of one kind (same G, first/last);
// group_of: each item's group index (device, n_items entries) or nullptr
// (the kernel then searches the groups' first_item prefix)
hipError_t launch_table(const EngineGroup* table, int n_groups, int n_items, const int* group_of, int G, bool first,
                        bool last, int rows, int in_t, int acc_t, hipStream_t s);
// direct quadrants (n <= 4) of a batch: n x W cells per group
hipError_t launch_table_direct(const EngineGroup* table, int n_groups, int n_items, int in_t, int acc_t,
                               hipStream_t s);
hipError_t launch_adjoint_pass(const AdjLaunch& L, int t, hipStream_t s);
hipError_t launch_adjoint_pair(const AdjLaunch& L, int t, hipStream_t s);
hipError_t launch_adjoint_direct(const AdjLaunch& L, int k, int t, hipStream_t s);
hipError_t launch_zero(void* p, int64_t rows, int64_t cols, int64_t ld, int elem_bytes, hipStream_t s);
hipError_t launch_shift(const void* in, int64_t ld_in, void* out, int64_t ld_out, int elem_bytes,
                        int hp, int wp, int inverse, hipStream_t s);
// Angle-range adjoint, last step: img[y, x] = a0[r, (c + sigma(r)) mod W]
// (r, c) = (y, x), or (x, y) when transposed; a0 is n x W, row pitch W.
hipError_t launch_unshear(const void* a0, int W, int n, int S1, void* img, int64_t ld_img, int w, int h,
                          int transposed, int elem_bytes, hipStream_t s);
int engine_grid_size();

// Launch timing (fht_timing_enable): the rocprof-style name of a pass kernel
// instantiation (in_t < 0: adjoint kernels, one type; op >= 0: the forward
// pass kernel's trailing operation argument), and the event pair
// around one launch.  timing_begin returns -1 when timing is off.
std::string kernel_name(const char* kernel, int in_t, int acc_t, int GB, bool first, bool last, int op = -1,
                        int nw = -1);
bool timing_on();
int timing_begin(const std::string& name, hipStream_t s);
void timing_end(int slot, hipStream_t s);

}  // namespace fht
