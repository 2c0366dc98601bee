// Host-side planning shared by the single-image and batched entry points.
#pragma once

#include "fht_internal.h"

#include <stddef.h>
#include <stdint.h>
#include <vector>

namespace fht {

// Pass structure and intermediate bands of one quadrant.  After pass p
// (j_end[p] stages) the nonzero columns of every row lie in a cyclic band of
// band_w[p] columns of the quadrant coordinate xi = dir * x; band index =
// (xi + band_off[p]) mod W.
struct QuadGeom {
    int q;           // 1..4
    int transposed;  // quadrants 3, 4 run on the transposed image
    int mirror;      // quadrants 2, 3 (dir = -1)
    int n;           // rows (h' or w')
    int other;       // the other padded side (w' or h')
    int W;
    int k;           // log2 n
    int npass;
    int G[4];        // stages per pass
    int j_end[4];
    int band_off[4];
    int band_w[4];
    int64_t band_ld[4];
    size_t band_byte_off[4];
};

int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int64_t pow2_ceil(int64_t v);
int ilog2(int64_t p);
void pass_split(int k, int* npass, int* G);
int tile_rows_for(int k, int G);
QuadGeom quad_geom(int w, int h, int q, int S1);
size_t quad_band_bytes(const QuadGeom& g, int p, int elem);
size_t layout_bands(QuadGeom* gs, int nq, int elem, size_t base);
int check_sides(int w, int h);
// Validates fht_forward's arguments (host only, no HIP call) and returns the
// workspace bytes the call needs in *need.
int forward_check(const void* img, int in_t, int w, int h, int64_t ld_img, const void* hough, int acc_t,
                  int64_t ld_hough, unsigned quads, unsigned flags, size_t* need);
int selected_quads(unsigned quads, int* qs);
void placement(int w, int h, unsigned quads, int q, int* base, int* sign, int* skip, int* roll_a, int* roll_b);
PassDesc make_pass_desc(const QuadGeom& g, int p, const void* img, int w, int h, int64_t ld_img, void* hough,
                        int64_t ld_hough, unsigned char* ws, int S1, int row_limit_final, int base, int sign,
                        int skip, int shifted, int roll_a, int roll_b);

// Engine groups of one image: pass p of quadrant i is emitted at step i + p
// (earlier passes first within a step), so a quadrant's next pass follows its
// previous one after one other quadrant's work; each group's dependency
// precedes it in the queue.  Quadrants with at most 2 stages (direct kernel)
// are not part of the engine.  Appends to out; returns the item count.
int append_engine_groups(const QuadGeom* gs, const PassDesc (*descs)[4], int nq, std::vector<EngineGroup>& out,
                         int first_item);

int engine_spin_limit();
int engine_agent_acquire();
int run_engine(const std::vector<EngineGroup>& groups, const EngineGroup* dev_table, int total_items,
               unsigned* sync, int in_t, int acc_t, hipStream_t stream);

}  // namespace fht
