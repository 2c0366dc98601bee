// Host AddressSanitizer / UndefinedBehaviorSanitizer run of the library's
// host side: shape and workspace queries, argument validation of every entry
// point (each call below is invalid and must be rejected before any HIP
// call, so no GPU is needed), the cell -> segment walk on every cell of small
// images, the pass-split table and the timing records.  Built from the host
// API units with the sanitizers on the host pass only, linked with the
// ordinary kernel objects; run by tests/test_sanitizers.py.
#include "fht.h"

#include <cstdint>
#include <cstdio>

static int fails = 0;
#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::printf("failed: %s (line %d)\n", #cond, __LINE__);         \
            ++fails;                                                        \
        }                                                                   \
    } while (0)

int main()
{
    int64_t r = 0, c = 0;
    size_t b = 0;
    const int sides[][2] = {{1, 1}, {3, 5}, {5, 3}, {64, 64}, {300, 520}, {65536, 5}, {5, 65536}};
    for (auto& s : sides) {
        const int w = s[0], h = s[1];
        for (unsigned q = 1; q <= 15; ++q) EXPECT(fht_hough_shape(w, h, q, &r, &c) == FHT_OK);
        for (int in_t = 0; in_t < 3; ++in_t) {
            const int acc = in_t == FHT_F32 ? FHT_F32 : FHT_I32;
            EXPECT(fht_workspace_size(w, h, FHT_FULL, in_t, acc, &b) == FHT_OK);
            EXPECT(fht_range_workspace_size(w, h, 0, 0, 0, in_t, acc, &b) == FHT_OK);
            EXPECT(fht_range_scaled_workspace_size(w, h, 3, 2, 0, 0, 1, in_t, acc, &b) == FHT_OK ||
                   w * 3 / 2 > FHT_MAX_SIDE || h * 3 / 2 > FHT_MAX_SIDE);
        }
        EXPECT(fht_adjoint_workspace_size(w, h, FHT_FULL, FHT_F32, &b) == FHT_OK);
        EXPECT(fht_adjoint_stack_workspace_size(w, h, FHT_FULL, FHT_F32, 7, &b) == FHT_OK);
    }
    EXPECT(fht_hough_shape(0, 5, FHT_FULL, &r, &c) == FHT_ERR_INVALID);
    EXPECT(fht_hough_shape(5, 5, 0, &r, &c) == FHT_ERR_INVALID);
    EXPECT(fht_hough_shape(5, 5, 16, &r, &c) == FHT_ERR_INVALID);
    EXPECT(fht_hough_shape(65537, 5, FHT_FULL, &r, &c) == FHT_ERR_INVALID);
    EXPECT(fht_hough_shape(5, 5, FHT_FULL, nullptr, &c) == FHT_ERR_INVALID);
    EXPECT(fht_range_shape(8, 8, 8, 3, 0, &r, &c) == FHT_ERR_INVALID);
    EXPECT(fht_range_shape(8, 8, 0, 8, 0, &r, &c) == FHT_ERR_INVALID);

    // invalid calls: rejected with a negative status before any HIP call
    void* p = reinterpret_cast<void*>(uintptr_t(1) << 20);
    fht_hough_shape(300, 200, FHT_FULL, &r, &c);
    EXPECT(fht_forward(nullptr, FHT_F32, 300, 200, 300, p, FHT_F32, c, FHT_FULL, 0, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_forward(p, FHT_U8, 300, 200, 300, p, FHT_F32, c, FHT_FULL, 0, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_forward(p, FHT_F32, 300, 200, 299, p, FHT_F32, c, FHT_FULL, 0, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_forward(p, FHT_F32, 300, 200, 300, p, FHT_F32, c - 1, FHT_FULL, 0, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_forward(p, FHT_F32, 300, 200, 300, p, FHT_F32, c, FHT_FULL, 64, p, 1u << 30, nullptr) < 0);
    {
        size_t sb = 0;
        EXPECT(fht_forward_stack_workspace_size(300, 200, FHT_FULL, FHT_F32, FHT_F32, 5, &sb) == FHT_OK && sb > 0);
        EXPECT(fht_forward_stack_workspace_size(300, 200, FHT_FULL, FHT_F32, FHT_F32, 0, &sb) < 0);
        EXPECT(fht_forward_stack(p, FHT_F32, 300, 200, 300, 300 * 200, 0, p, FHT_F32, c, r * c, FHT_FULL, 0, p, sb,
                                 nullptr) < 0);
        EXPECT(fht_forward_stack(p, FHT_F32, 300, 200, 300, 300 * 200 - 1, 5, p, FHT_F32, c, r * c, FHT_FULL, 0, p,
                                 sb, nullptr) < 0);
        EXPECT(fht_forward_stack(p, FHT_F32, 300, 200, 300, 300 * 200, 5, p, FHT_F32, c, r * c - 1, FHT_FULL, 0, p,
                                 sb, nullptr) < 0);
        EXPECT(fht_forward_stack(p, FHT_F32, 300, 200, 300, 300 * 200, 5, p, FHT_F32, c, r * c, FHT_FULL, 0, p,
                                 sb - 1, nullptr) < 0);
    }
    EXPECT(fht_forward(p, FHT_F32, 300, 200, 300, p, FHT_F32, c, FHT_Q1, FHT_FLAG_SHIFTED, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_forward(p, FHT_F32, 300, 200, 300, p, FHT_F32, c, FHT_FULL, 0, p, 16, nullptr) == FHT_ERR_WORKSPACE);
    EXPECT(fht_forward(p, FHT_F32, 300, 200, 300, p, FHT_F32, c, FHT_FULL, 0, (char*)p + 4, 1u << 30, nullptr) < 0);
    // the allocation-free forward: the same validation, then the scratch limit, before any HIP call
    EXPECT(fht_forward_noalloc(nullptr, FHT_F32, 300, 200, 300, p, FHT_F32, c, FHT_FULL, 0, nullptr) < 0);
    EXPECT(fht_forward_noalloc(p, FHT_F32, 300, 200, 299, p, FHT_F32, c, FHT_FULL, 0, nullptr) < 0);
    EXPECT(fht_forward_noalloc(p, FHT_F32, 2048, 2048, 2048, p, FHT_F32, 4096, FHT_FULL, 0, nullptr) ==
           FHT_ERR_UNSUPPORTED);
    EXPECT(fht_engine_status(nullptr, nullptr) == FHT_ERR_INVALID);
    EXPECT(fht_set_tile_rows(10, 48) == FHT_ERR_INVALID);
    EXPECT(fht_set_tile_rows(2, 32) == FHT_ERR_INVALID);
    EXPECT(fht_range(p, FHT_F32, 300, 200, 300, 300, 2, 0, p, FHT_F32, c, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_range(p, FHT_F32, 300, 200, 300, 2, 2, 0, p, FHT_I32, c, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_range_scaled(p, FHT_F32, 300, 200, 300, 0, 1, 0, 0, 0, p, FHT_F32, c, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_range_adjoint(p, FHT_U8, c, 0, 0, 0, p, 300, 300, 200, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_shift(p, c, p, c, FHT_F32, 300, 200, 0, nullptr) < 0);                   // in place needs W*4 small
    EXPECT(fht_shift((char*)p + 64, c, p, c, FHT_F32, 300, 200, 0, nullptr) < 0);       // partial overlap
    EXPECT(fht_shift(p, c - 1, (char*)p + (1u << 30), c, FHT_F32, 300, 200, 0, nullptr) < 0);
    EXPECT(fht_adjoint(p, FHT_F32, c, p, 300, 300, 200, FHT_FULL, FHT_FLAG_MAX, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_adjoint(p, FHT_F32, c, p, 299, 300, 200, FHT_FULL, 0, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_adjoint(p, FHT_F32, c, p, 300, 300, 200, FHT_FULL, 0, p, 16, nullptr) == FHT_ERR_WORKSPACE);
    EXPECT(fht_adjoint_stack(p, FHT_F32, c, r * c - 1, p, 300, 300 * 200, 300, 200, 3, FHT_FULL, 0, p, 1u << 30,
                             nullptr) < 0);
    EXPECT(fht_peaks(p, FHT_F32, 10, 10, 10, 0, 0.0, (int64_t*)p, 10, (unsigned*)p, nullptr) < 0);
    EXPECT(fht_peaks(p, FHT_U8, 10, 10, 10, 1, 0.0, (int64_t*)p, 10, (unsigned*)p, nullptr) < 0);
    const int32_t ws1[2] = {64, 0}, hs1[2] = {64, 64};
    fht_batch_plan* plan = nullptr;
    int64_t tot = 0;
    EXPECT(fht_batch_plan_create(ws1, hs1, 2, FHT_FULL, FHT_U8, FHT_I32, &plan, &b, &tot, nullptr) < 0);
    EXPECT(fht_batch_plan_create(ws1, hs1, 0, FHT_FULL, FHT_U8, FHT_I32, &plan, &b, &tot, nullptr) < 0);
    EXPECT(fht_batch_plan_create(nullptr, hs1, 1, FHT_FULL, FHT_U8, FHT_I32, &plan, &b, &tot, nullptr) < 0);
    EXPECT(fht_batch_forward(nullptr, nullptr, p, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_batch_forward_stack(nullptr, p, 64, p, p, 1u << 30, nullptr) < 0);
    EXPECT(fht_batch_plan_destroy(nullptr) == FHT_OK);
    for (int st = -6; st <= 0; ++st) EXPECT(fht_status_string(st) != nullptr);
    EXPECT(fht_last_error() != nullptr);

    // cell -> segment on every cell of small images
    const int small[][2] = {{1, 1}, {5, 7}, {16, 12}, {13, 32}};
    for (auto& s : small) {
        const int w = s[0], h = s[1];
        fht_hough_shape(w, h, FHT_FULL, &r, &c);
        int32_t seg[5];
        for (int64_t row = 0; row < r; ++row)
            for (int64_t x0 = 0; x0 < c; ++x0) {
                EXPECT(fht_cell_segment(w, h, FHT_FULL, row, x0, 0, seg) == FHT_OK);
                EXPECT(fht_cell_segment(w, h, FHT_FULL, row, x0, 1, seg) == FHT_OK);
            }
        EXPECT(fht_cell_segment(w, h, FHT_FULL, r, 0, 0, seg) < 0);
        EXPECT(fht_cell_segment(w, h, FHT_FULL, 0, c, 0, seg) < 0);
    }

    // pass splits, timing records
    int np = 0, g[4];
    for (int side = 1; side <= 65536; side *= 2) EXPECT(fht_pass_split(side, &np, g) == FHT_OK);
    const int split[2] = {5, 6};
    EXPECT(fht_set_pass_split(11, 2, split) == FHT_OK);
    EXPECT(fht_pass_split(2048, &np, g) == FHT_OK && np == 2 && g[0] == 5 && g[1] == 6);
    EXPECT(fht_set_pass_split(11, 0, nullptr) == FHT_OK);
    const int bad[2] = {2, 9};
    EXPECT(fht_set_pass_split(11, 2, bad) < 0);
    EXPECT(fht_timing_filter("pass") == FHT_OK);
    EXPECT(fht_timing_filter(nullptr) == FHT_OK);
    char name[64];
    int64_t launches = 0;
    double ms = 0;
    EXPECT(fht_timing_report(0, name, sizeof name, &launches, &ms) == FHT_ERR_INVALID);

    std::printf("library host sanitizer run: %s\n", fails ? "FAILED" : "clean");
    return fails ? 1 : 0;
}
