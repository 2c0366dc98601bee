// C ABI of libfht.so (declared in include/fht.h): argument validation, pass
// planning, workspace layout and launch orchestration.  All arithmetic runs in
// the kernels of fht_device.h.

#include "fht.h"
#include "fht_internal.h"
#include "fht_plan.h"

#include <mutex>
#include <vector>

#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace fht {

static thread_local char g_last_error[512] = "";

int fail(int status, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return status;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(FHT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int64_t pow2_ceil(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

int ilog2(int64_t p)
{
    int k = 0;
    while ((int64_t(1) << k) < p) ++k;
    return k;
}

// Stage-fusion split: k stages in ceil(k/6) passes of 3..6 stages (k <= 2
// runs as one direct pass).
// Stage split per k, set by fht_set_pass_split / fht_autotune (npass 0:
// the default rule).  Read at planning time only.
static std::mutex g_split_mu;
static int g_split[32][5];
// tile height per k for passes of at most 5 stages (0: the default rule),
// set by fht_set_tile_rows / fht_autotune; guarded by g_split_mu
static int g_rows[32];

// Tile height of a pass of G stages of a quadrant with 2^k rows.  Passes of
// 6 stages need 64-row tiles.  Otherwise 32 unless set for k: twice the
// tiles and four workgroups per CU measured faster at every size tried
// (side 128 to 2048, uint8 and float32: 3 to 15 %; the 512-image batch 4 %).
int tile_rows_for(int k, int G)
{
    if (G > 5) return kTileRows;
    std::lock_guard<std::mutex> lock(g_split_mu);
    if (k >= 0 && k < 32 && g_rows[k] > 0) return g_rows[k];
    return kNarrowRows;
}

static int default_passes(int k) { return (k + kMaxG - 1) / kMaxG; }

void pass_split(int k, int* npass, int* G)
{
    if (k <= 2) {
        *npass = 1;
        G[0] = k;
        return;
    }
    {
        std::lock_guard<std::mutex> lock(g_split_mu);
        if (k < 32 && g_split[k][0] > 0) {
            *npass = g_split[k][0];
            for (int i = 0; i < *npass; ++i) G[i] = g_split[k][1 + i];
            return;
        }
    }
    // Fewest passes of at most kMaxG stages.  Two passes: the first as deep
    // as it can be (the last keeps at least 3 stages).  Measured on MI355X
    // against the even split: equal or faster on single images (256^2 to
    // 1024^2, uint8 and float32: forward within 3 %, the 512^2 adjoint 10 %)
    // and 5-6 % on the 16 x 1024^2 stack and the 512-image batch.  Three or
    // more passes: as even as possible, larger first (8192^2: the deepest
    // first pass, 6+4+3, was 3 % slower than 5+4+4).
    const int np = default_passes(k);
    if (np == 2) {
        G[0] = k - 3 < kMaxG ? k - 3 : kMaxG;
        G[1] = k - G[0];
    } else {
        const int base = k / np, rem = k % np;
        for (int i = 0; i < np; ++i) G[i] = base + (i < rem ? 1 : 0);
    }
    *npass = np;
}

// Every split of k into the fewest passes of 3..kMaxG stages.
static std::vector<std::vector<int>> split_candidates(int k)
{
    std::vector<std::vector<int>> out;
    const int np = default_passes(k);
    std::vector<int> cur(np, 3);
    for (;;) {
        int sum = 0;
        for (int g : cur) sum += g;
        if (sum == k) out.push_back(cur);
        int i = np - 1;
        while (i >= 0 && cur[i] == kMaxG) cur[i--] = 3;
        if (i < 0) break;
        ++cur[i];
    }
    return out;
}

// Geometry of quadrant q (1..4) of an h x w image; S1 != 0 adds the range shear
// (unmirrored quadrants only).
QuadGeom quad_geom(int w, int h, int q, int S1)
{
    QuadGeom g{};
    const int hp = (int)pow2_ceil(h), wp = (int)pow2_ceil(w);
    g.q = q;
    g.transposed = q >= 3;
    g.mirror = (q == 2 || q == 3) ? 1 : 0;
    g.n = g.transposed ? wp : hp;
    g.other = g.transposed ? hp : wp;
    g.W = hp + wp;
    g.k = ilog2(g.n);
    pass_split(g.k, &g.npass, g.G);
    int j = 0;
    for (int p = 0; p < g.npass; ++p) {
        j += g.G[p];
        g.j_end[p] = j;
        // nonzero columns after j stages, in xi: unmirrored, the image columns
        // moved by the shear (rows roll right by 0..S1) and widened by 2^j - 1
        // towards negative xi; mirrored, x in [0, other + 2^j - 1) i.e.
        // xi in [-(other + 2^j - 2), 0]
        const int64_t spread = (int64_t(1) << j) - 1;
        int64_t lo, hi;
        if (!g.mirror) {
            lo = (S1 < 0 ? S1 : 0) - spread;
            hi = (S1 > 0 ? S1 : 0) + g.other;
        } else {
            lo = -(g.other + spread - 1);
            hi = 1;
        }
        // band origin on a 64-column boundary keeps the tile windows aligned
        lo = -(((-lo) + 63) / 64) * 64;
        int64_t bw = hi - lo;
        if (bw > g.W) bw = g.W;
        g.band_off[p] = (int)(-lo);
        g.band_w[p] = (int)bw;
        g.band_ld[p] = (bw + 63) / 64 * 64;
    }
    return g;
}

size_t quad_band_bytes(const QuadGeom& g, int p, int elem)
{
    return ((size_t)g.n * (size_t)g.band_ld[p] * (size_t)elem + 255) / 256 * 256;
}

// Lays out the intermediate bands of the selected quadrants after `base`
// bytes; returns the end offset.
size_t layout_bands(QuadGeom* gs, int nq, int elem, size_t base)
{
    size_t off = base;
    for (int i = 0; i < nq; ++i)
        for (int p = 0; p + 1 < gs[i].npass; ++p) {
            gs[i].band_byte_off[p] = off;
            off += quad_band_bytes(gs[i], p, elem);
        }
    return off;
}

static bool dtype_pair_ok(int in_t, int acc_t)
{
    return (in_t == FHT_U8 && acc_t == FHT_I32) || (in_t == FHT_I32 && acc_t == FHT_I32) ||
           (in_t == FHT_F32 && acc_t == FHT_F32);
}

static int elem_size(int t) { return t == FHT_U8 ? 1 : 4; }

int check_sides(int w, int h)
{
    if (w < 1 || h < 1) return fail(FHT_ERR_INVALID, "image sides must be >= 1 (got w=%d h=%d)", w, h);
    if (pow2_ceil(w) > FHT_MAX_SIDE || pow2_ceil(h) > FHT_MAX_SIDE)
        return fail(FHT_ERR_INVALID, "padded side exceeds %d", FHT_MAX_SIDE);
    return FHT_OK;
}

int selected_quads(unsigned quads, int* qs)
{
    int nq = 0;
    for (int q = 1; q <= 4; ++q)
        if (quads & (1u << (q - 1))) qs[nq++] = q;
    return nq;
}

// Hough row placement of quadrant q's shift s.
void placement(int w, int h, unsigned quads, int q, int* base, int* sign, int* skip, int* roll_a, int* roll_b)
{
    const int hp = (int)pow2_ceil(h), wp = (int)pow2_ceil(w);
    *roll_a = (q <= 2) ? hp : wp;
    *roll_b = (q == 1 || q == 4) ? 1 : -1;
    if (quads == FHT_FULL) {
        // section 3.3: flip(H1); H2[1:]; flip(H3)[1:]; H4[1:]
        switch (q) {
        case 1: *base = hp - 1; *sign = -1; *skip = -1; break;
        case 2: *base = hp - 1; *sign = 1; *skip = 0; break;
        case 3: *base = 2 * hp + wp - 3; *sign = -1; *skip = wp - 1; break;
        default: *base = 2 * hp + wp - 3; *sign = 1; *skip = 0; break;
        }
        return;
    }
    int off = 0;
    for (int p = 1; p < q; ++p)
        if (quads & (1u << (p - 1))) off += (p <= 2) ? hp : wp;
    *base = off;
    *sign = 1;
    *skip = -1;
}

// Descriptor of forward pass p of quadrant geometry g.
PassDesc make_pass_desc(const QuadGeom& g, int p, const void* img, int w, int h, int64_t ld_img, void* hough,
                        int64_t ld_hough, unsigned char* ws, int S1, int row_limit_final, int base, int sign,
                        int skip, int shifted, int roll_a, int roll_b)
{
    PassDesc d{};
    const int G = g.G[p];
    const int VW = kWinCols - (1 << G);
    d.n = g.n;
    d.W = g.W;
    d.j0 = p == 0 ? 0 : g.j_end[p - 1];
    d.G = G;
    d.mirror = g.mirror;
    d.img_w = w;
    d.img_h = h;
    d.tile_rows = tile_rows_for(g.k, G);
    d.n_row_tiles = (g.n + d.tile_rows - 1) / d.tile_rows;
    if (p == 0) {
        d.src = img;
        d.src_ld = ld_img;
        d.src_kind = g.transposed ? SRC_IMAGE_T : SRC_IMAGE;
        d.S1 = S1;
    } else {
        d.src = ws + g.band_byte_off[p - 1];
        d.src_ld = g.band_ld[p - 1];
        d.src_kind = SRC_BAND;
        d.src_off = g.band_off[p - 1];
        d.src_bw = g.band_w[p - 1];
    }
    if (p == g.npass - 1) {
        d.dst = hough;
        d.dst_ld = ld_hough;
        d.dst_kind = DST_HOUGH;
        // mirrored: the lane's run of xi = 8l + 1 .. 8l + 8 maps to x = -xi,
        // a run starting on an 8-column (32-byte) boundary; unaligned vector
        // stores cost about 1.7x as much
        d.x_start = g.mirror ? 1 : 0;
        d.n_windows = (g.W + VW - 1) / VW;
        d.row_limit = row_limit_final;
        d.row_base = base;
        d.row_sign = sign;
        d.skip_row = skip;
        d.shifted = shifted;
        d.roll_a = roll_a;
        d.roll_b = roll_b;
        // black zone of row s (section 3.2): xi in [other, other + n - s)
        // unmirrored, [1, 1 + n - s) mirrored; not with a shear
        d.black_lo = g.mirror ? 1 : g.other;
        d.black_ok = (S1 == 0) ? 1 : 0;
    } else {
        d.dst = ws + g.band_byte_off[p];
        d.dst_ld = g.band_ld[p];
        d.dst_kind = DST_BAND;
        d.dst_off = g.band_off[p];
        d.dst_bw = g.band_w[p];
        d.x_start = -g.band_off[p];
        d.n_windows = (g.band_w[p] + VW - 1) / VW;
        d.row_limit = row_limit_final == INT_MAX ? INT_MAX : (row_limit_final >> (g.k - g.j_end[p]));
        d.skip_row = -1;
    }
    return d;
}

int append_engine_groups(const QuadGeom* gs, const PassDesc (*descs)[4], int nq, std::vector<EngineGroup>& out,
                         int first_item)
{
    int maxp = 0;
    for (int i = 0; i < nq; ++i)
        if (gs[i].k > 2 && gs[i].npass > maxp) maxp = gs[i].npass;
    int group_of[4][4];
    int item = first_item;
    for (int step = 0; step < nq + maxp; ++step) {
        for (int p = 0; p < maxp; ++p) {
            const int i = step - p;
            if (i < 0 || i >= nq || gs[i].k <= 2 || p >= gs[i].npass) continue;
            EngineGroup e{};
            e.d = descs[i][p];
            // the engine runs 64-row tiles only
            e.d.tile_rows = kTileRows;
            e.d.n_row_tiles = (e.d.n + kTileRows - 1) / kTileRows;
            e.first_item = item;
            e.count = e.d.n_row_tiles * e.d.n_windows;
            e.dep = p > 0 ? group_of[i][p - 1] : -1;
            e.dep_count = p > 0 ? out[group_of[i][p - 1]].count : 0;
            e.notify = p + 1 < gs[i].npass ? 1 : 0;
            group_of[i][p] = (int)out.size();
            out.push_back(e);
            item += e.count;
        }
    }
    return item - first_item;
}

// Iterations of the bounded dependency wait (each sleeps ~256 cycles plus
// the atomic's round trip): far beyond any legitimate wait, short enough that
// a planner error ends the launch within seconds, with word 1 of the
// workspace set to nonzero (the engine's error flag) instead of a hang.
int engine_spin_limit()
{
    static int lim = -1;
    if (lim < 0) {
        const char* e = getenv("FHT_SPIN_LIMIT");
        lim = e ? atoi(e) : (1 << 21);
        if (lim < 1) lim = 1;
    }
    return lim;
}

// Launches the engine over `groups` (queue order, dependencies pointing
// backwards).  Groups of different depth G run in separate launches, deepest
// first: a quadrant's passes have non-increasing depth, so a dependency on a
// group of another depth is on an earlier launch and stream order covers it.
// FHT_ACQUIRE=0 selects the light acquire after a dependency wait (see
// wait_group); the default is the agent-scope acquire.
int engine_agent_acquire()
{
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("FHT_ACQUIRE");
        v = (e && e[0] == '0') ? 0 : 1;
    }
    return v;
}

int run_engine(const std::vector<EngineGroup>& groups, const EngineGroup* dev_table, int total_items,
               unsigned* sync, int in_t, int acc_t, hipStream_t stream)
{
    (void)total_items;
    (void)dev_table;
    if (groups.empty()) return FHT_OK;
    const int grid_max = engine_grid_size();
    // word 1 (the error flag) is cleared once per call, so a wait that gave
    // up in an earlier launch of the call stays visible to fht_engine_status
    hipError_t ez = launch_zero(sync + 1, 1, 1, 1, 4, stream);
    if (ez != hipSuccess) return hip_fail(ez, "engine error flag reset");
    for (int G = kMaxG; G >= 3; --G) {
        std::vector<int> remap(groups.size(), -1);
        EngineArgs A{};
        int item = 0;
        int n = 0;
        for (size_t i = 0; i < groups.size(); ++i) {
            if (groups[i].d.G != G) continue;
            if (n >= kEngineInline) return fail(FHT_ERR_UNSUPPORTED, "too many engine groups of one depth");
            EngineGroup e = groups[i];
            e.first_item = item;
            e.dep = (e.dep >= 0 && remap[e.dep] >= 0) ? remap[e.dep] : -1;
            remap[i] = n;
            A.g[n++] = e;
            item += e.count;
        }
        if (n == 0) continue;
        A.n_groups = n;
        A.total_items = item;
        A.sync = sync;
        A.spin_limit = engine_spin_limit();
        A.agent_acquire = engine_agent_acquire();
        A.table = nullptr;
        // queue head (word 0) and the group counters (words 2..n+1)
        hipError_t e = launch_zero(sync, 1, 1, 1, 4, stream);
        if (e == hipSuccess) e = launch_zero(sync + 2, 1, n, n, 4, stream);
        if (e != hipSuccess) return hip_fail(e, "engine counter reset");
        e = launch_engine(A, G, item < grid_max ? item : grid_max, in_t, acc_t, stream);
        if (e != hipSuccess) return hip_fail(e, "engine launch");
    }
    return FHT_OK;
}

// FHT_ENGINE=1 selects the persistent engine instead of one launch per pass.
static bool use_engine()
{
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("FHT_ENGINE");
        v = (e && e[0] == '1') ? 1 : 0;
    }
    return v == 1;
}

// Runs the forward passes of the quadrant geometries gs[0..nq).
// op: 0 = sum along the patterns, 1 = max.
// m > 1: a stack of m images, the descriptors' steps giving image i's
// buffers; every launch covers all m (never the engine).
static int run_forward(const QuadGeom* gs, const PassDesc (*descs)[4], int nq, int in_t, int acc_t, unsigned* sync,
                       hipStream_t stream, int op = 0, int m = 1)
{
    // quadrants with at most two stages: one direct launch
    for (int i = 0; i < nq; ++i) {
        if (gs[i].k > 2) continue;
        PassLaunch L{};
        L.d[0] = descs[i][0];
        L.nd = 1;
        L.n_img = m;
        hipError_t e = launch_direct(L, gs[i].k, in_t, acc_t, stream, op);
        if (e != hipSuccess) return hip_fail(e, "direct launch");
    }
    bool sheared = false;
    for (int i = 0; i < nq; ++i) sheared |= descs[i][0].S1 != 0 || descs[i][0].scale_num != 0;
    // the engine runs unsheared, unscaled sources only; the angle range
    // always takes the per-pass launches
    if (use_engine() && op == 0 && !sheared && m == 1) {
        std::vector<EngineGroup> groups;
        const int total = append_engine_groups(gs, descs, nq, groups, 0);
        return run_engine(groups, nullptr, total, sync, in_t, acc_t, stream);
    }
    int maxp = 0;
    for (int i = 0; i < nq; ++i) maxp = gs[i].npass > maxp ? gs[i].npass : maxp;
    for (int p = 0; p < maxp; ++p) {
        for (int G = kMaxG; G >= 3; --G) {
            for (int last = 0; last < 2; ++last) {
                for (int rows = kTileRows; rows >= kNarrowRows; rows /= 2) {
                    PassLaunch L{};
                    L.n_img = m;
                    for (int i = 0; i < nq; ++i)
                        if (gs[i].k > 2 && p < gs[i].npass && gs[i].G[p] == G &&
                            (p == gs[i].npass - 1) == (last == 1) && descs[i][p].tile_rows == rows)
                            L.d[L.nd++] = descs[i][p];
                    if (L.nd == 0) continue;
                    const int ti = p == 0 ? in_t : acc_t;
                    hipError_t e = launch_pass(L, ti, acc_t, stream, op);
                    if (e != hipSuccess) return hip_fail(e, "forward pass launch");
                }
            }
        }
    }
    return FHT_OK;
}

// Workspace: engine counters, then the intermediate bands.
static size_t forward_workspace(QuadGeom* gs, int nq, int acc_t)
{
    int groups = 0;
    for (int i = 0; i < nq; ++i)
        if (gs[i].k > 2) groups += gs[i].npass;
    return layout_bands(gs, nq, elem_size(acc_t), engine_sync_bytes(groups));
}

}  // namespace fht

using namespace fht;

extern "C" {

int fht_version(void) { return 10100; }

const char* fht_status_string(int status)
{
    switch (status) {
    case FHT_OK: return "ok";
    case FHT_ERR_INVALID: return "invalid argument";
    case FHT_ERR_UNSUPPORTED: return "unsupported request";
    case FHT_ERR_WORKSPACE: return "workspace missing or too small";
    case FHT_ERR_HIP: return "HIP runtime error";
    case FHT_ERR_TIMEOUT: return "dependency wait timed out";
    default: return "unknown status";
    }
}

const char* fht_last_error(void) { return g_last_error; }

int fht_pass_split(int side, int* npass, int* passes)
{
    if (!npass || !passes) return fail(FHT_ERR_INVALID, "null output");
    if (side < 1 || pow2_ceil(side) > FHT_MAX_SIDE) return fail(FHT_ERR_INVALID, "bad side %d", side);
    int G[4];
    pass_split(ilog2(pow2_ceil(side)), npass, G);
    for (int i = 0; i < *npass; ++i) passes[i] = G[i];
    return FHT_OK;
}

int fht_engine_status(const void* workspace, void* stream)
{
    if (!workspace) return fail(FHT_ERR_INVALID, "null workspace");
    unsigned flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, (const unsigned char*)workspace + 4, sizeof flag, hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "reading the engine's error flag");
    if (flag) return fail(FHT_ERR_TIMEOUT, "a dependency wait of the persistent engine gave up; the results of that call "
                                           "are invalid");
    return FHT_OK;
}

int fht_set_tile_rows(int k, int rows)
{
    if (k < 3 || k > 16) return fail(FHT_ERR_INVALID, "k %d outside 3..16", k);
    if (rows != 0 && rows != kTileRows && rows != kNarrowRows)
        return fail(FHT_ERR_INVALID, "tile rows %d: 0 (default), %d or %d", rows, kNarrowRows, kTileRows);
    std::lock_guard<std::mutex> lock(g_split_mu);
    g_rows[k] = rows;
    return FHT_OK;
}

int fht_tile_rows(int side, int* rows)
{
    if (!rows) return fail(FHT_ERR_INVALID, "null output");
    if (side < 1 || pow2_ceil(side) > FHT_MAX_SIDE) return fail(FHT_ERR_INVALID, "bad side %d", side);
    *rows = tile_rows_for(ilog2(pow2_ceil(side)), 5);
    return FHT_OK;
}

int fht_set_pass_split(int k, int npass, const int* passes)
{
    if (k < 3 || k > 16) return fail(FHT_ERR_INVALID, "k %d outside 3..16", k);
    if (npass == 0) {
        std::lock_guard<std::mutex> lock(g_split_mu);
        g_split[k][0] = 0;
        return FHT_OK;
    }
    if (!passes) return fail(FHT_ERR_INVALID, "null passes");
    if (npass != default_passes(k))
        return fail(FHT_ERR_INVALID, "k = %d takes %d passes, not %d", k, default_passes(k), npass);
    int sum = 0;
    for (int i = 0; i < npass; ++i) {
        if (passes[i] < 3 || passes[i] > kMaxG) return fail(FHT_ERR_INVALID, "pass of %d stages", passes[i]);
        sum += passes[i];
    }
    if (sum != k) return fail(FHT_ERR_INVALID, "stages sum to %d, not %d", sum, k);
    std::lock_guard<std::mutex> lock(g_split_mu);
    g_split[k][0] = npass;
    for (int i = 0; i < npass; ++i) g_split[k][1 + i] = passes[i];
    return FHT_OK;
}

int fht_autotune(int w, int h, int in_t, int acc_t, int reps, void* stream)
{
    int rc = check_sides(w, h);
    if (rc) return rc;
    if (!dtype_pair_ok(in_t, acc_t)) return fail(FHT_ERR_INVALID, "unsupported dtype pair (%d, %d)", in_t, acc_t);
    if (reps < 1 || reps > 1000) return fail(FHT_ERR_INVALID, "reps %d outside 1..1000", reps);
    const int kh = ilog2(pow2_ceil(h)), kw = ilog2(pow2_ceil(w));
    // candidates per stage count: every split into the fewest passes, each
    // with 64-row tiles and, when some pass has at most 5 stages, 32-row tiles
    struct Cfg {
        std::vector<int> split;
        int rows;
    };
    auto candidates = [](int k) {
        std::vector<Cfg> out;
        for (auto& sp : split_candidates(k)) {
            out.push_back({sp, kTileRows});
            bool narrow_ok = false;
            for (int g : sp) narrow_ok |= g <= 5;
            if (narrow_ok) out.push_back({sp, kNarrowRows});
        }
        return out;
    };
    auto apply = [](int k, const Cfg& c) {
        fht_set_pass_split(k, (int)c.split.size(), c.split.data());
        fht_set_tile_rows(k, c.rows);
    };
    std::vector<int> ks;
    for (int k : {kh, kw})
        if (k >= 3 && candidates(k).size() > 1 && (ks.empty() || ks[0] != k)) ks.push_back(k);
    if (ks.empty()) return FHT_OK;
    const std::vector<Cfg> ca = candidates(ks[0]);
    const std::vector<Cfg> cb = ks.size() > 1 ? candidates(ks[1]) : std::vector<Cfg>{Cfg{{}, 0}};
    // buffers for the largest workspace over every combination
    size_t ws_max = 0;
    for (auto& a : ca)
        for (auto& b : cb) {
            apply(ks[0], a);
            if (ks.size() > 1) apply(ks[1], b);
            size_t need = 0;
            fht_workspace_size(w, h, FHT_FULL, in_t, acc_t, &need);
            ws_max = need > ws_max ? need : ws_max;
        }
    int64_t rows, cols;
    fht_hough_shape(w, h, FHT_FULL, &rows, &cols);
    const size_t in_bytes = (size_t)w * h * (in_t == FHT_U8 ? 1 : 4);
    void *img = nullptr, *hough = nullptr, *ws = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMalloc(&img, in_bytes);
    if (e == hipSuccess) e = hipMalloc(&hough, (size_t)rows * cols * 4);
    if (e == hipSuccess) e = hipMalloc(&ws, ws_max > 256 ? ws_max : 256);
    if (e == hipSuccess) e = hipMemsetAsync(img, 0, in_bytes, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = -1.f;
    Cfg best_a, best_b;
    for (auto& a : ca) {
        for (auto& b : cb) {
            if (e != hipSuccess) break;
            apply(ks[0], a);
            if (ks.size() > 1) apply(ks[1], b);
            rc = fht_forward(img, in_t, w, h, w, hough, acc_t, cols, FHT_FULL, 0, ws, ws_max > 256 ? ws_max : 256,
                             stream);  // warm-up
            if (rc) break;
            if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
            for (int r = 0; r < reps && rc == FHT_OK; ++r)
                rc = fht_forward(img, in_t, w, h, w, hough, acc_t, cols, FHT_FULL, 0, ws,
                                 ws_max > 256 ? ws_max : 256, stream);
            if (rc) break;
            if ((e = hipEventRecord(e1, s)) != hipSuccess) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (best < 0.f || ms < best) {
                best = ms;
                best_a = a;
                best_b = b;
            }
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipStreamSynchronize(s);
    hipFree(img);
    hipFree(hough);
    hipFree(ws);
    // keep the fastest (or the default rules if timing failed)
    for (int k : ks) {
        fht_set_pass_split(k, 0, nullptr);
        fht_set_tile_rows(k, 0);
    }
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (rc) return rc;
    apply(ks[0], best_a);
    if (ks.size() > 1) apply(ks[1], best_b);
    return FHT_OK;
}

int fht_hough_shape(int w, int h, unsigned quads, int64_t* rows, int64_t* cols)
{
    if (!rows || !cols) return fail(FHT_ERR_INVALID, "null shape output");
    int rc = check_sides(w, h);
    if (rc) return rc;
    if (quads == 0 || (quads & ~15u)) return fail(FHT_ERR_INVALID, "bad quadrant selection 0x%x", quads);
    const int64_t hp = pow2_ceil(h), wp = pow2_ceil(w);
    *cols = hp + wp;
    if (quads == FHT_FULL) {
        *rows = 2 * (hp + wp) - 3;
    } else {
        int64_t r = 0;
        for (int q = 1; q <= 4; ++q)
            if (quads & (1u << (q - 1))) r += (q <= 2) ? hp : wp;
        *rows = r;
    }
    return FHT_OK;
}

int fht_range_shape(int w, int h, int S1, int S, int transposed, int64_t* rows, int64_t* cols)
{
    if (!rows || !cols) return fail(FHT_ERR_INVALID, "null shape output");
    int rc = check_sides(w, h);
    if (rc) return rc;
    const int64_t hp = pow2_ceil(h), wp = pow2_ceil(w);
    const int64_t n = transposed ? wp : hp;
    if (S < 0 || S > n - 1) return fail(FHT_ERR_INVALID, "S=%d outside [0, %lld]", S, (long long)(n - 1));
    if (S1 > n - 1 || S1 < -(n - 1)) return fail(FHT_ERR_INVALID, "|S1|=%d exceeds %lld", S1, (long long)(n - 1));
    *rows = (int64_t)S + 1;
    *cols = hp + wp;
    return FHT_OK;
}

int fht_workspace_size(int w, int h, unsigned quads, int in_t, int acc_t, size_t* bytes)
{
    if (!bytes) return fail(FHT_ERR_INVALID, "null bytes output");
    int64_t r, c;
    int rc = fht_hough_shape(w, h, quads, &r, &c);
    if (rc) return rc;
    if (!dtype_pair_ok(in_t, acc_t)) return fail(FHT_ERR_INVALID, "unsupported dtype pair (%d, %d)", in_t, acc_t);
    int qs[4];
    const int nq = selected_quads(quads, qs);
    QuadGeom gs[4];
    for (int i = 0; i < nq; ++i) gs[i] = quad_geom(w, h, qs[i], 0);
    *bytes = forward_workspace(gs, nq, acc_t);
    return FHT_OK;
}

// Adjoint workspace: the bands.  The image passes add their contributions
// to the image gradient itself, in quadrant order (run_adjoint).
static size_t adjoint_workspace(QuadGeom* gs, int nq) { return layout_bands(gs, nq, 4, 0); }

int fht_adjoint_workspace_size(int w, int h, unsigned quads, int t, size_t* bytes)
{
    if (!bytes) return fail(FHT_ERR_INVALID, "null bytes output");
    if (t != FHT_I32 && t != FHT_F32) return fail(FHT_ERR_INVALID, "adjoint type must be I32 or F32");
    int64_t r, c;
    int rc = fht_hough_shape(w, h, quads, &r, &c);
    if (rc) return rc;
    int qs[4];
    const int nq = selected_quads(quads, qs);
    QuadGeom gs[4];
    for (int i = 0; i < nq; ++i) gs[i] = quad_geom(w, h, qs[i], 0);
    *bytes = adjoint_workspace(gs, nq);
    return FHT_OK;
}

int fht_range_workspace_size(int w, int h, int S1, int S, int transposed, int in_t, int acc_t, size_t* bytes)
{
    if (!bytes) return fail(FHT_ERR_INVALID, "null bytes output");
    int64_t r, c;
    int rc = fht_range_shape(w, h, S1, S, transposed, &r, &c);
    if (rc) return rc;
    if (!dtype_pair_ok(in_t, acc_t)) return fail(FHT_ERR_INVALID, "unsupported dtype pair (%d, %d)", in_t, acc_t);
    QuadGeom g = quad_geom(w, h, transposed ? 4 : 1, S1);
    *bytes = forward_workspace(&g, 1, acc_t);
    return FHT_OK;
}

}  // extern "C"

namespace fht {

int forward_check(const void* img, int in_t, int w, int h, int64_t ld_img, const void* hough, int acc_t,
                  int64_t ld_hough, unsigned quads, unsigned flags, size_t* need)
{
    int64_t rows, cols;
    int rc = fht_hough_shape(w, h, quads, &rows, &cols);
    if (rc) return rc;
    if (!img || !hough) return fail(FHT_ERR_INVALID, "null image or Hough pointer");
    if (!dtype_pair_ok(in_t, acc_t)) return fail(FHT_ERR_INVALID, "unsupported dtype pair (%d, %d)", in_t, acc_t);
    if (ld_img < w) return fail(FHT_ERR_INVALID, "ld_img %lld < w %d", (long long)ld_img, w);
    if (ld_hough < cols) return fail(FHT_ERR_INVALID, "ld_hough %lld < %lld", (long long)ld_hough, (long long)cols);
    if (flags & ~(unsigned)(FHT_FLAG_SHIFTED | FHT_FLAG_MAX)) return fail(FHT_ERR_INVALID, "unknown flags 0x%x", flags);
    if ((flags & FHT_FLAG_SHIFTED) && quads != FHT_FULL)
        return fail(FHT_ERR_INVALID, "fhtshift applies to the full Hough image only");
    int qs[4];
    const int nq = selected_quads(quads, qs);
    QuadGeom gs[4];
    for (int i = 0; i < nq; ++i) gs[i] = quad_geom(w, h, qs[i], 0);
    *need = forward_workspace(gs, nq, acc_t);
    return FHT_OK;
}

}  // namespace fht

extern "C" {

int fht_forward(const void* img, int in_t, int w, int h, int64_t ld_img, void* hough, int acc_t, int64_t ld_hough,
                unsigned quads, unsigned flags, void* workspace, size_t ws_bytes, void* stream)
{
    size_t need = 0;
    int rc = forward_check(img, in_t, w, h, ld_img, hough, acc_t, ld_hough, quads, flags, &need);
    if (rc) return rc;
    int qs[4];
    const int nq = selected_quads(quads, qs);
    QuadGeom gs[4];
    for (int i = 0; i < nq; ++i) gs[i] = quad_geom(w, h, qs[i], 0);
    forward_workspace(gs, nq, acc_t);  // lays out the bands in gs
    if (!workspace || ws_bytes < need)
        return fail(FHT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    if ((uintptr_t)workspace & 255) return fail(FHT_ERR_INVALID, "workspace must be 256-byte aligned");
    PassDesc descs[4][4];
    for (int i = 0; i < nq; ++i) {
        int base, sign, skip, ra, rb;
        placement(w, h, quads, qs[i], &base, &sign, &skip, &ra, &rb);
        for (int p = 0; p < gs[i].npass; ++p)
            descs[i][p] = make_pass_desc(gs[i], p, img, w, h, ld_img, hough, ld_hough, (unsigned char*)workspace, 0,
                                         INT_MAX, base, sign, skip, (flags & FHT_FLAG_SHIFTED) ? 1 : 0, ra, rb);
    }
    return run_forward(gs, descs, nq, in_t, acc_t, (unsigned*)workspace, (hipStream_t)stream,
                       (flags & FHT_FLAG_MAX) ? 1 : 0);
}

// Images of a forward stack per group: their bands within 8 GiB (the batch
// plan's chunk), at most 65535 (the launch grid's y extent).
static int forward_stack_group(size_t slice, int n)
{
    const size_t budget = size_t(8) << 30;
    size_t g = slice ? budget / slice : (size_t)n;
    if (g > 65535) g = 65535;
    if (g > (size_t)n) g = (size_t)n;
    return g < 1 ? 1 : (int)g;
}

int fht_forward_stack_workspace_size(int w, int h, unsigned quads, int in_t, int acc_t, int n, size_t* bytes)
{
    if (!bytes) return fail(FHT_ERR_INVALID, "null bytes output");
    if (n < 1) return fail(FHT_ERR_INVALID, "stack of %d images", n);
    size_t one = 0;
    int rc = fht_workspace_size(w, h, quads, in_t, acc_t, &one);
    if (rc) return rc;
    const size_t slice = (one + 255) / 256 * 256;
    *bytes = (size_t)forward_stack_group(slice, n) * slice;
    return FHT_OK;
}

int fht_forward_stack(const void* img, int in_t, int w, int h, int64_t ld_img, int64_t img_stride, int n, void* hough,
                      int acc_t, int64_t ld_hough, int64_t hough_stride, unsigned quads, unsigned flags,
                      void* workspace, size_t ws_bytes, void* stream)
{
    size_t one = 0;
    int rc = forward_check(img, in_t, w, h, ld_img, hough, acc_t, ld_hough, quads, flags, &one);
    if (rc) return rc;
    if (n < 1) return fail(FHT_ERR_INVALID, "stack of %d images", n);
    int64_t rows, cols;
    fht_hough_shape(w, h, quads, &rows, &cols);
    if (n > 1 && img_stride < (int64_t)h * ld_img)
        return fail(FHT_ERR_INVALID, "img_stride %lld < h * ld_img", (long long)img_stride);
    if (n > 1 && hough_stride < rows * ld_hough)
        return fail(FHT_ERR_INVALID, "hough_stride %lld < rows * ld_hough", (long long)hough_stride);
    const size_t slice = (one + 255) / 256 * 256;
    const int group = forward_stack_group(slice, n);
    const size_t need = (size_t)group * slice;
    if (!workspace || ws_bytes < need)
        return fail(FHT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    if ((uintptr_t)workspace & 255) return fail(FHT_ERR_INVALID, "workspace must be 256-byte aligned");
    int qs[4];
    const int nq = selected_quads(quads, qs);
    QuadGeom gs[4];
    for (int i = 0; i < nq; ++i) gs[i] = quad_geom(w, h, qs[i], 0);
    forward_workspace(gs, nq, acc_t);  // lays out the bands in gs
    const int64_t img_step = img_stride * (int64_t)elem_size(in_t);
    const int64_t hough_step = hough_stride * (int64_t)elem_size(acc_t);
    for (int i0 = 0; i0 < n; i0 += group) {
        const int m = n - i0 < group ? n - i0 : group;
        const unsigned char* im0 = (const unsigned char*)img + (int64_t)i0 * img_step;
        unsigned char* h0 = (unsigned char*)hough + (int64_t)i0 * hough_step;
        PassDesc descs[4][4];
        for (int i = 0; i < nq; ++i) {
            int base, sign, skip, ra, rb;
            placement(w, h, quads, qs[i], &base, &sign, &skip, &ra, &rb);
            for (int p = 0; p < gs[i].npass; ++p) {
                PassDesc& d = descs[i][p];
                d = make_pass_desc(gs[i], p, im0, w, h, ld_img, h0, ld_hough, (unsigned char*)workspace, 0, INT_MAX,
                                   base, sign, skip, (flags & FHT_FLAG_SHIFTED) ? 1 : 0, ra, rb);
                d.src_step = p == 0 ? img_step : (int64_t)slice;
                d.dst_step = p == gs[i].npass - 1 ? hough_step : (int64_t)slice;
            }
        }
        rc = run_forward(gs, descs, nq, in_t, acc_t, (unsigned*)workspace, (hipStream_t)stream,
                         (flags & FHT_FLAG_MAX) ? 1 : 0, m);
        if (rc) return rc;
    }
    return FHT_OK;
}

int fht_range(const void* img, int in_t, int w, int h, int64_t ld_img, int S1, int S, int transposed, void* hough,
              int acc_t, int64_t ld_hough, void* workspace, size_t ws_bytes, void* stream)
{
    int64_t rows, cols;
    int rc = fht_range_shape(w, h, S1, S, transposed, &rows, &cols);
    if (rc) return rc;
    if (!img || !hough) return fail(FHT_ERR_INVALID, "null image or Hough pointer");
    if (!dtype_pair_ok(in_t, acc_t)) return fail(FHT_ERR_INVALID, "unsupported dtype pair (%d, %d)", in_t, acc_t);
    if (ld_img < w) return fail(FHT_ERR_INVALID, "ld_img %lld < w %d", (long long)ld_img, w);
    if (ld_hough < cols) return fail(FHT_ERR_INVALID, "ld_hough %lld < %lld", (long long)ld_hough, (long long)cols);
    QuadGeom g = quad_geom(w, h, transposed ? 4 : 1, S1);
    const size_t need = forward_workspace(&g, 1, acc_t);
    if (!workspace || ws_bytes < need)
        return fail(FHT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    if ((uintptr_t)workspace & 255) return fail(FHT_ERR_INVALID, "workspace must be 256-byte aligned");
    PassDesc descs[1][4];
    for (int p = 0; p < g.npass; ++p)
        descs[0][p] = make_pass_desc(g, p, img, w, h, ld_img, hough, ld_hough, (unsigned char*)workspace, S1, S, 0, 1,
                                     -1, 0, 0, 0);
    return run_forward(&g, descs, 1, in_t, acc_t, (unsigned*)workspace, (hipStream_t)stream);
}

// Scaled angle range (section 4): the scaled image has ceil(extent * num /
// den) samples along the sheared axis (columns; rows when transposed).
static int scaled_sizes(int w, int h, int num, int den, int transposed, int* ws, int* hs)
{
    if (num < 1 || den < 1 || num > 64 || den > 64)
        return fail(FHT_ERR_INVALID, "scale %d/%d: numerator and denominator in 1..64", num, den);
    const int64_t a = transposed ? h : w;
    const int64_t sc = (a * num + den - 1) / den;
    if (sc > FHT_MAX_SIDE) return fail(FHT_ERR_UNSUPPORTED, "scaled side %lld exceeds %d", (long long)sc, FHT_MAX_SIDE);
    *ws = transposed ? w : (int)sc;
    *hs = transposed ? (int)sc : h;
    return FHT_OK;
}

int fht_range_scaled_shape(int w, int h, int num, int den, int S1, int S, int transposed, int64_t* rows,
                           int64_t* cols)
{
    int rc = check_sides(w, h);
    if (rc) return rc;
    int ws, hs;
    rc = scaled_sizes(w, h, num, den, transposed, &ws, &hs);
    if (rc) return rc;
    return fht_range_shape(ws, hs, S1, S, transposed, rows, cols);
}

int fht_range_scaled_workspace_size(int w, int h, int num, int den, int S1, int S, int transposed, int in_t,
                                    int acc_t, size_t* bytes)
{
    int rc = check_sides(w, h);
    if (rc) return rc;
    int ws, hs;
    rc = scaled_sizes(w, h, num, den, transposed, &ws, &hs);
    if (rc) return rc;
    return fht_range_workspace_size(ws, hs, S1, S, transposed, in_t, acc_t, bytes);
}

int fht_range_scaled(const void* img, int in_t, int w, int h, int64_t ld_img, int num, int den, int S1, int S,
                     int transposed, void* hough, int acc_t, int64_t ld_hough, void* workspace, size_t ws_bytes,
                     void* stream)
{
    int rc = check_sides(w, h);
    if (rc) return rc;
    int ws, hs;
    rc = scaled_sizes(w, h, num, den, transposed, &ws, &hs);
    if (rc) return rc;
    int64_t rows, cols;
    rc = fht_range_shape(ws, hs, S1, S, transposed, &rows, &cols);
    if (rc) return rc;
    if (!img || !hough) return fail(FHT_ERR_INVALID, "null image or Hough pointer");
    if (!dtype_pair_ok(in_t, acc_t)) return fail(FHT_ERR_INVALID, "unsupported dtype pair (%d, %d)", in_t, acc_t);
    if (ld_img < w) return fail(FHT_ERR_INVALID, "ld_img %lld < w %d", (long long)ld_img, w);
    if (ld_hough < cols) return fail(FHT_ERR_INVALID, "ld_hough %lld < %lld", (long long)ld_hough, (long long)cols);
    QuadGeom g = quad_geom(ws, hs, transposed ? 4 : 1, S1);
    const size_t need = forward_workspace(&g, 1, acc_t);
    if (!workspace || ws_bytes < need)
        return fail(FHT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    if ((uintptr_t)workspace & 255) return fail(FHT_ERR_INVALID, "workspace must be 256-byte aligned");
    PassDesc descs[1][4];
    for (int p = 0; p < g.npass; ++p) {
        // the descriptors see the scaled extents; the first pass maps a
        // scaled sample back to its source sample
        descs[0][p] = make_pass_desc(g, p, img, ws, hs, ld_img, hough, ld_hough, (unsigned char*)workspace, S1, S, 0,
                                     1, -1, 0, 0, 0);
        if (p == 0 && num != den) {
            descs[0][p].scale_num = num;
            descs[0][p].scale_den = den;
        }
    }
    return run_forward(&g, descs, 1, in_t, acc_t, (unsigned*)workspace, (hipStream_t)stream);
}

int fht_shift(const void* in, int64_t ld_in, void* out, int64_t ld_out, int t, int w, int h, int inverse, void* stream)
{
    int rc = check_sides(w, h);
    if (rc) return rc;
    if (!in || !out) return fail(FHT_ERR_INVALID, "null pointer");
    if (t != FHT_I32 && t != FHT_F32) return fail(FHT_ERR_INVALID, "fht_shift type must be I32 or F32");
    const int64_t hp = pow2_ceil(h), wp = pow2_ceil(w), W = hp + wp, rows = 2 * (hp + wp) - 3;
    if (ld_in < W || ld_out < W) return fail(FHT_ERR_INVALID, "pitch smaller than W=%lld", (long long)W);
    const char* a0 = (const char*)in;
    const char* a1 = a0 + (size_t)((rows - 1) * ld_in + W) * 4;
    const char* b0 = (const char*)out;
    const char* b1 = b0 + (size_t)((rows - 1) * ld_out + W) * 4;
    const bool same = (in == out) && ld_in == ld_out;
    if (!same && a0 < b1 && b0 < a1) return fail(FHT_ERR_INVALID, "in and out overlap without being identical");
    if (same && W * 4 > 163840) return fail(FHT_ERR_UNSUPPORTED, "in-place fhtshift needs W*4 <= 163840");
    hipError_t e = launch_shift(in, ld_in, out, ld_out, 4, (int)hp, (int)wp, inverse ? 1 : 0, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fht_shift launch");
    return FHT_OK;
}

}  // extern "C"

namespace fht {

AdjDesc make_adj_desc(const QuadGeom& g, int p, const void* grad, int64_t ld_grad, void* gimg, int64_t ld_img, int w,
                      int h, unsigned char* ws, int base, int sign, int skip, int shifted, int roll_a, int roll_b,
                      int accumulate)
{
    AdjDesc d{};
    const int G = g.G[p];
    const int VW = kWinCols - (1 << G);
    d.row_limit = INT_MAX;  // every Hough row is read (angle range: set to S)
    d.n = g.n;
    d.W = g.W;
    d.j0 = p == 0 ? 0 : g.j_end[p - 1];
    d.G = G;
    d.mirror = g.mirror;
    d.img_w = w;
    d.img_h = h;
    d.n_row_tiles = (g.n + kTileRows - 1) / kTileRows;
    if (p == g.npass - 1) {
        d.src = grad;
        d.src_ld = ld_grad;
        d.src_kind = 0;
        d.row_base = base;
        d.row_sign = sign;
        d.skip_row = skip;
        d.shifted = shifted;
        d.roll_a = roll_a;
        d.roll_b = roll_b;
        // the gradient on the zone of section 3.2 (case c) reaches only the
        // zero padding, never an image pixel, so it is read as zero: the
        // image gradient does not change, not even in rounding (every sum
        // that reaches an image pixel has the same terms)
        d.black_lo = g.mirror ? 1 : g.other;
        d.black_ok = 1;
    } else {
        d.src = ws + g.band_byte_off[p];
        d.src_ld = g.band_ld[p];
        d.src_kind = 1;
        d.src_off = g.band_off[p];
        d.src_bw = g.band_w[p];
        d.skip_row = -1;
    }
    if (p == 0) {
        d.dst = gimg;
        d.dst_ld = ld_img;
        d.dst_kind = g.transposed ? 2 : 1;
        d.accumulate = accumulate;
        // image columns 0..cols-1 are xi = x (unmirrored) or xi = W - x (mirrored)
        const int cols = g.transposed ? h : w;
        d.x_start = g.mirror ? g.W - cols + 1 : 0;
        d.n_windows = (cols + VW - 1) / VW;
    } else {
        d.dst = ws + g.band_byte_off[p - 1];
        d.dst_ld = g.band_ld[p - 1];
        d.dst_kind = 0;
        d.dst_off = g.band_off[p - 1];
        d.dst_bw = g.band_w[p - 1];
        d.x_start = 0;
        d.n_windows = (g.W + VW - 1) / VW;
    }
    return d;
}

// Adjoint of a stack of same-size images in one set of launches: image i's
// gradient, output and workspace slice (its bands) sit i * grad_step,
// i * img_step and i * ws_step bytes after image 0's; the launches run the
// image index on their z axis.
struct AdjStack {
    const void* grad;
    void* img;
    unsigned char* ws;
    int64_t grad_step, img_step, ws_step;
    int m;
};

// Images per stack group: their bands within 2 GiB, at most 8192 (the grid's
// z extent, 4 descriptors per image, stays below 2^15).
static int stack_group(size_t slice, int n)
{
    const size_t budget = size_t(2) << 30;
    size_t g = slice ? budget / slice : (size_t)n;
    if (g > 8192) g = 8192;
    if (g > (size_t)n) g = (size_t)n;
    return g < 1 ? 1 : (int)g;
}

int check_adjoint_args(const void* grad_hough, int t, int64_t ld_hough, const void* grad_img, int64_t ld_img, int w,
                       int h, unsigned quads, unsigned flags)
{
    int64_t rows, cols;
    int rc = fht_hough_shape(w, h, quads, &rows, &cols);
    if (rc) return rc;
    if (!grad_hough || !grad_img) return fail(FHT_ERR_INVALID, "null gradient pointer");
    if (t != FHT_I32 && t != FHT_F32) return fail(FHT_ERR_INVALID, "adjoint type must be I32 or F32");
    if (ld_img < w) return fail(FHT_ERR_INVALID, "ld_img %lld < w %d", (long long)ld_img, w);
    if (ld_hough < cols) return fail(FHT_ERR_INVALID, "ld_hough %lld < %lld", (long long)ld_hough, (long long)cols);
    if (flags & FHT_FLAG_MAX) return fail(FHT_ERR_INVALID, "the adjoint is the transpose of the sum transform");
    if (flags & ~(unsigned)FHT_FLAG_SHIFTED) return fail(FHT_ERR_INVALID, "unknown flags 0x%x", flags);
    if ((flags & FHT_FLAG_SHIFTED) && quads != FHT_FULL)
        return fail(FHT_ERR_INVALID, "fhtshift applies to the full Hough image only");
    return FHT_OK;
}

int run_adjoint(const AdjStack& S, int t, int64_t ld_hough, int64_t ld_img, int w, int h, unsigned quads,
                unsigned flags, hipStream_t s)
{
    int qs[4];
    const int nq = selected_quads(quads, qs);
    QuadGeom gs[4];
    for (int i = 0; i < nq; ++i) gs[i] = quad_geom(w, h, qs[i], 0);
    layout_bands(gs, nq, 4, 0);  // each quadrant's band offsets in the workspace
    // Image passes in steps, in quadrant order: a mirror pair (quadrants 1
    // and 2, or 3 and 4, both with pass kernels), whose tiles one workgroup
    // computes together, or one quadrant.  The first step stores its values
    // in the image gradient; every later one adds its own to what is stored
    // there, so the image receives ((q1 + q2) + q3) + q4, the contributions
    // in quadrant order (a pair's kernel adds the mirrored member's values
    // first: (s + q3) + q4).
    struct Step {
        int u, m;  // pair: unmirrored and mirrored quadrant indices; single: u, m = -1
    };
    Step steps[4];
    int n_steps = 0;
    for (int i = 0; i < nq;) {
        if (i + 1 < nq && (qs[i] == 1 || qs[i] == 3) && qs[i + 1] == qs[i] + 1 && gs[i].k > 2 && gs[i + 1].k > 2) {
            // quadrant 1 and 4 are unmirrored, 2 and 3 mirrored
            steps[n_steps++] = qs[i] == 1 ? Step{i, i + 1} : Step{i + 1, i};
            i += 2;
        } else {
            steps[n_steps++] = Step{i, -1};
            i += 1;
        }
    }
    AdjDesc descs[4][4];
    for (int i = 0; i < nq; ++i) {
        int base, sign, skip, ra, rb;
        placement(w, h, quads, qs[i], &base, &sign, &skip, &ra, &rb);
        for (int p = 0; p < gs[i].npass; ++p) {
            AdjDesc& d = descs[i][p];
            d = make_adj_desc(gs[i], p, S.grad, ld_hough, S.img, ld_img, w, h, S.ws, base, sign, skip,
                              (flags & FHT_FLAG_SHIFTED) ? 1 : 0, ra, rb, 0);
            d.src_step = p == gs[i].npass - 1 ? S.grad_step : S.ws_step;
            d.dst_step = p == 0 ? S.img_step : S.ws_step;
        }
    }
    for (int st = 1; st < n_steps; ++st) {
        const int members[2] = {steps[st].u, steps[st].m};
        for (int i : members)
            if (i >= 0) descs[i][0].accumulate = 1;
    }
    int maxp = 0;
    for (int i = 0; i < nq; ++i) maxp = gs[i].npass > maxp ? gs[i].npass : maxp;
    // band passes (p >= 1) in reverse order, every quadrant's pass of one
    // kind in one launch over the stack
    for (int p = maxp - 1; p >= 1; --p) {
        for (int G = 3; G <= kMaxG; ++G) {
            for (int first = 0; first < 2; ++first) {
                AdjLaunch L{};
                L.n_img = S.m;
                for (int i = 0; i < nq; ++i)
                    if (gs[i].k > 2 && p < gs[i].npass && gs[i].G[p] == G && (p == gs[i].npass - 1) == (first == 1))
                        L.d[L.nd++] = descs[i][p];
                if (L.nd == 0) continue;
                hipError_t e = launch_adjoint_pass(L, t, s);
                if (e != hipSuccess) return hip_fail(e, "adjoint pass launch");
            }
        }
    }
    // the image-pass steps, each once the previous one has stored
    for (int st = 0; st < n_steps; ++st) {
        const Step& P = steps[st];
        AdjLaunch L{};
        L.n_img = S.m;
        L.d[L.nd++] = descs[P.u][0];
        hipError_t e;
        if (P.m >= 0) {
            L.d[L.nd++] = descs[P.m][0];
            e = launch_adjoint_pair(L, t, s);
        } else {
            e = gs[P.u].k > 2 ? launch_adjoint_pass(L, t, s) : launch_adjoint_direct(L, gs[P.u].k, t, s);
        }
        if (e != hipSuccess) return hip_fail(e, "adjoint image pass launch");
    }
    return FHT_OK;
}

}  // namespace fht

extern "C" {

int fht_adjoint(const void* grad_hough, int t, int64_t ld_hough, void* grad_img, int64_t ld_img, int w, int h,
                unsigned quads, unsigned flags, void* workspace, size_t ws_bytes, void* stream)
{
    int rc = check_adjoint_args(grad_hough, t, ld_hough, grad_img, ld_img, w, h, quads, flags);
    if (rc) return rc;
    int qs[4];
    const int nq = selected_quads(quads, qs);
    QuadGeom gs[4];
    for (int i = 0; i < nq; ++i) gs[i] = quad_geom(w, h, qs[i], 0);
    const size_t need = adjoint_workspace(gs, nq);
    if (need > 0 && (!workspace || ws_bytes < need))
        return fail(FHT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    if (workspace && ((uintptr_t)workspace & 255)) return fail(FHT_ERR_INVALID, "workspace must be 256-byte aligned");
    const AdjStack S{grad_hough, grad_img, (unsigned char*)workspace, 0, 0, 0, 1};
    return run_adjoint(S, t, ld_hough, ld_img, w, h, quads, flags, (hipStream_t)stream);
}

int fht_adjoint_stack_workspace_size(int w, int h, unsigned quads, int t, int n, size_t* bytes)
{
    if (!bytes) return fail(FHT_ERR_INVALID, "null bytes output");
    if (n < 1) return fail(FHT_ERR_INVALID, "stack of %d images", n);
    size_t one = 0;
    int rc = fht_adjoint_workspace_size(w, h, quads, t, &one);
    if (rc) return rc;
    const size_t slice = (one + 255) / 256 * 256;
    *bytes = (size_t)stack_group(slice, n) * slice;
    return FHT_OK;
}

int fht_adjoint_stack(const void* grad_hough, int t, int64_t ld_hough, int64_t grad_stride, void* grad_img,
                      int64_t ld_img, int64_t img_stride, int w, int h, int n, unsigned quads, unsigned flags,
                      void* workspace, size_t ws_bytes, void* stream)
{
    int rc = check_adjoint_args(grad_hough, t, ld_hough, grad_img, ld_img, w, h, quads, flags);
    if (rc) return rc;
    if (n < 1) return fail(FHT_ERR_INVALID, "stack of %d images", n);
    int64_t rows, cols;
    fht_hough_shape(w, h, quads, &rows, &cols);
    if (n > 1 && grad_stride < rows * ld_hough)
        return fail(FHT_ERR_INVALID, "grad_stride %lld < rows * ld_hough", (long long)grad_stride);
    if (n > 1 && img_stride < (int64_t)h * ld_img)
        return fail(FHT_ERR_INVALID, "img_stride %lld < h * ld_img", (long long)img_stride);
    size_t need = 0;
    rc = fht_adjoint_stack_workspace_size(w, h, quads, t, n, &need);
    if (rc) return rc;
    if (!workspace || ws_bytes < need)
        return fail(FHT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    if ((uintptr_t)workspace & 255) return fail(FHT_ERR_INVALID, "workspace must be 256-byte aligned");
    size_t one = 0;
    fht_adjoint_workspace_size(w, h, quads, t, &one);
    const size_t slice = (one + 255) / 256 * 256;
    const int group = stack_group(slice, n);
    const size_t esz = 4;
    for (int i0 = 0; i0 < n; i0 += group) {
        AdjStack S;
        S.grad = (const unsigned char*)grad_hough + (size_t)i0 * (size_t)grad_stride * esz;
        S.img = (unsigned char*)grad_img + (size_t)i0 * (size_t)img_stride * esz;
        S.ws = (unsigned char*)workspace;
        S.grad_step = grad_stride * (int64_t)esz;
        S.img_step = img_stride * (int64_t)esz;
        S.ws_step = (int64_t)slice;
        S.m = n - i0 < group ? n - i0 : group;
        rc = run_adjoint(S, t, ld_hough, ld_img, w, h, quads, flags, (hipStream_t)stream);
        if (rc) return rc;
    }
    return FHT_OK;
}

// Angle-range adjoint: the bands of the range's quadrant geometry, then the
// n x W gradient of the sheared padded source.
static size_t range_adjoint_workspace(QuadGeom& g)
{
    const size_t bands = layout_bands(&g, 1, 4, 0);
    return bands + ((size_t)g.n * (size_t)g.W * 4 + 255) / 256 * 256;
}

int fht_range_adjoint_workspace_size(int w, int h, int S1, int S, int transposed, int t, size_t* bytes)
{
    if (!bytes) return fail(FHT_ERR_INVALID, "null bytes output");
    if (t != FHT_I32 && t != FHT_F32) return fail(FHT_ERR_INVALID, "adjoint type must be I32 or F32");
    int64_t r, c;
    int rc = fht_range_shape(w, h, S1, S, transposed, &r, &c);
    if (rc) return rc;
    QuadGeom g = quad_geom(w, h, transposed ? 4 : 1, S1);
    *bytes = range_adjoint_workspace(g);
    return FHT_OK;
}

int fht_range_adjoint(const void* grad, int t, int64_t ld_grad, int S1, int S, int transposed, void* grad_img,
                      int64_t ld_img, int w, int h, void* workspace, size_t ws_bytes, void* stream)
{
    int64_t rows, cols;
    int rc = fht_range_shape(w, h, S1, S, transposed, &rows, &cols);
    if (rc) return rc;
    if (!grad || !grad_img) return fail(FHT_ERR_INVALID, "null gradient pointer");
    if (t != FHT_I32 && t != FHT_F32) return fail(FHT_ERR_INVALID, "adjoint type must be I32 or F32");
    if (ld_img < w) return fail(FHT_ERR_INVALID, "ld_img %lld < w %d", (long long)ld_img, w);
    if (ld_grad < cols) return fail(FHT_ERR_INVALID, "ld_grad %lld < %lld", (long long)ld_grad, (long long)cols);
    QuadGeom g = quad_geom(w, h, transposed ? 4 : 1, S1);
    const size_t need = range_adjoint_workspace(g);
    if (!workspace || ws_bytes < need)
        return fail(FHT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? ws_bytes : 0);
    if ((uintptr_t)workspace & 255) return fail(FHT_ERR_INVALID, "workspace must be 256-byte aligned");
    unsigned char* ws = (unsigned char*)workspace;
    unsigned char* a0 = ws + layout_bands(&g, 1, 4, 0);
    hipStream_t s = (hipStream_t)stream;
    // passes in reverse order; the one reading the gradient reads rows 0..S,
    // the last one writes the full-width source gradient a0 (n x W)
    for (int p = g.npass - 1; p >= 0; --p) {
        AdjDesc d = make_adj_desc(g, p, grad, ld_grad, nullptr, 0, w, h, ws, 0, 1, -1, 0, 0, 0, 0);
        if (p == g.npass - 1) {
            d.row_limit = S;
            d.black_ok = 0;  // the zone moves with the shear
        }
        if (p == 0) {
            const int VW = kWinCols - (1 << g.G[0]);
            d.dst = a0;
            d.dst_ld = g.W;
            d.dst_kind = 0;
            d.dst_off = 0;
            d.dst_bw = g.W;
            d.accumulate = 0;
            d.x_start = 0;
            d.n_windows = (g.W + VW - 1) / VW;
        }
        AdjLaunch L{};
        L.d[0] = d;
        L.nd = 1;
        hipError_t e = g.k <= 2 ? launch_adjoint_direct(L, g.k, t, s) : launch_adjoint_pass(L, t, s);
        if (e != hipSuccess) return hip_fail(e, "range adjoint pass launch");
    }
    hipError_t e = launch_unshear(a0, g.W, g.n, S1, grad_img, ld_img, w, h, transposed, 4, s);
    if (e != hipSuccess) return hip_fail(e, "range adjoint unshear launch");
    return FHT_OK;
}

}  // extern "C"
