// Host-side planning shared by the single-image and batched entry points.
#pragma once

#include "fht_internal.h"

#include <stddef.h>
#include <stdint.h>

namespace fht {

// Pass structure and intermediate bands of one quadrant.  After pass p
// (j_end[p] stages) the nonzero columns of every row lie in a cyclic band of
// band_w[p] columns; band index = (x + band_off[p]) mod W.
struct QuadGeom {
    int q;           // 1..4
    int transposed;  // quadrants 3, 4 run on the transposed image
    int n;           // rows (h' or w')
    int other;       // the other padded side (w' or h')
    int W;
    int k;           // log2 n
    int dir;         // +1 or -1
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
QuadGeom quad_geom(int w, int h, int q, int S1);
size_t quad_band_bytes(const QuadGeom& g, int p, int elem);
size_t layout_bands(QuadGeom* gs, int nq, int elem);
int check_sides(int w, int h);
int selected_quads(unsigned quads, int* qs);
void placement(int w, int h, unsigned quads, int q, int* base, int* sign, int* skip, int* roll_a, int* roll_b);
PassDesc make_pass_desc(const QuadGeom& g, int p, const void* img, int in_src_kind, int w, int h,
                        int64_t ld_img, void* hough, int64_t ld_hough, unsigned char* ws, int S1,
                        int row_limit_final, int base, int sign, int skip, int shifted, int roll_a,
                        int roll_b);

}  // namespace fht
