// Batched forward over many images of different sizes (fht_batch_* in fht.h).
//
// A plan lays out, once, every pass of every quadrant of every image as an
// engine group whose pointers are byte offsets: image index, offset in the
// packed Hough buffer, offset in the workspace.  A call copies the template
// into the workspace with the pointers resolved (one small kernel), then runs
// one table-driven launch per (pass, depth, last-pass, tile height) class: every tile of
// every image of that class in one grid.  Images are processed in chunks
// whose intermediate bands fit a fixed budget, so the workspace stays
// bounded; chunks follow each other on the stream.  Everything enqueued is a
// kernel, so a call can be captured in a hipGraph.

#include "fht.h"
#include "fht_internal.h"
#include "fht_plan.h"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace fht {

constexpr size_t kBatchBandBudget = size_t(8) << 30;  // bytes of bands per chunk
constexpr int64_t kBatchMapItems = int64_t(1) << 26;   // item -> group map entries (256 MB) at most

struct BatchLaunch {
    int first_group;  // index into the table
    int n_groups;
    int n_items;
    int64_t map_off;  // tile launches: the launch's item -> group map in the plan's map; -1: none
    int G;
    int rows;         // tile height of the class (64 or 32)
    bool first, last;
};

struct BatchTemplate {
    int img;          // image index (image sources)
    int src_is_ws;    // src offset is into the workspace (band), else image
    int dst_is_ws;    // dst offset is into the workspace (band), else the Hough buffer
    int pad_;
    int64_t src_off;  // bytes
    int64_t dst_off;  // bytes
};

// Copies the template table into the workspace with pointers resolved.
// Image i is imgs[i], or with imgs == nullptr base + i * stride (bytes).
__global__ void fht_batch_fixup_kernel(const EngineGroup* __restrict__ tmpl, const BatchTemplate* __restrict__ rel,
                                       int n_groups, const void* const* imgs, const unsigned char* base,
                                       int64_t stride, unsigned char* hough, unsigned char* ws, EngineGroup* out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    EngineGroup e = tmpl[g];
    const BatchTemplate r = rel[g];
    const void* img = imgs ? imgs[r.img] : (const void*)(base + (int64_t)r.img * stride);
    e.d.src = r.src_is_ws ? (const void*)(ws + r.src_off) : img;
    e.d.dst = r.dst_is_ws ? (void*)(ws + r.dst_off) : (void*)(hough + r.dst_off);
    out[g] = e;
}

}  // namespace fht

struct fht_batch_plan {
    int n = 0;
    unsigned quads = 0;
    int in_t = 0, acc_t = 0;
    int device = 0;
    std::vector<int32_t> ws, hs;
    std::vector<int64_t> out_off;
    int64_t out_elems = 0;
    size_t table_bytes = 0;   // resolved table at the start of the workspace
    size_t ws_bytes = 0;
    int n_groups = 0;
    std::vector<fht::BatchLaunch> launches;  // in stream order (chunks, passes, classes)
    fht::EngineGroup* d_tmpl = nullptr;
    fht::BatchTemplate* d_rel = nullptr;
    int* d_map = nullptr;  // item -> group (relative to the launch's first group) of every tile launch
};

using namespace fht;

extern "C" {

int fht_batch_plan_create(const int32_t* ws, const int32_t* hs, int n, unsigned quads, int in_t, int acc_t,
                          fht_batch_plan** plan, size_t* ws_bytes, int64_t* out_elems, int64_t* out_offsets)
{
    if (!ws || !hs || !plan || !ws_bytes || !out_elems || n < 1) return fail(FHT_ERR_INVALID, "bad batch arguments");
    *plan = nullptr;
    if (!((in_t == FHT_U8 && acc_t == FHT_I32) || (in_t == FHT_I32 && acc_t == FHT_I32) ||
          (in_t == FHT_F32 && acc_t == FHT_F32)))
        return fail(FHT_ERR_INVALID, "unsupported dtype pair (%d, %d)", in_t, acc_t);
    if (quads == 0 || (quads & ~15u)) return fail(FHT_ERR_INVALID, "bad quadrant selection 0x%x", quads);
    for (int i = 0; i < n; ++i) {
        int rc = check_sides(ws[i], hs[i]);
        if (rc) return rc;
    }
    fht_batch_plan* P = new fht_batch_plan();
    P->n = n;
    P->quads = quads;
    P->in_t = in_t;
    P->acc_t = acc_t;
    P->ws.assign(ws, ws + n);
    P->hs.assign(hs, hs + n);
    hipGetDevice(&P->device);

    // output layout: image after image, each dense (ld = W_i)
    P->out_off.resize(n);
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        int64_t r, c;
        fht_hough_shape(ws[i], hs[i], quads, &r, &c);
        P->out_off[i] = off;
        off += r * c;
    }
    P->out_elems = off;
    const int esz = 4;

    // per image geometry and descriptors (pointers as offsets)
    int qs[4];
    const int nq = selected_quads(quads, qs);
    std::vector<EngineGroup> tmpl;
    std::vector<BatchTemplate> rel;
    size_t band_peak = 0;
    // chunks of images with bounded band memory
    int i0 = 0;
    while (i0 < n) {
        size_t band = 0;
        int i1 = i0;
        std::vector<QuadGeom> geoms;
        while (i1 < n) {
            QuadGeom gs[4];
            for (int q = 0; q < nq; ++q) gs[q] = quad_geom(ws[i1], hs[i1], qs[q], 0);
            const size_t b = layout_bands(gs, nq, esz, 0);
            if (i1 > i0 && band + b > kBatchBandBudget) break;
            for (int q = 0; q < nq; ++q) {
                for (int p = 0; p + 1 < gs[q].npass; ++p) gs[q].band_byte_off[p] += band;
                geoms.push_back(gs[q]);
            }
            band += b;
            ++i1;
        }
        band_peak = std::max(band_peak, band);
        // groups of this chunk, by (pass, depth, last, tile height)
        struct Item { EngineGroup e; BatchTemplate r; int p, G, last, rows; };
        std::vector<Item> items;
        for (int i = i0; i < i1; ++i) {
            for (int q = 0; q < nq; ++q) {
                const QuadGeom& g = geoms[(size_t)(i - i0) * nq + q];
                int base, sign, skip, ra, rb;
                placement(ws[i], hs[i], quads, qs[q], &base, &sign, &skip, &ra, &rb);
                int64_t r, c;
                fht_hough_shape(ws[i], hs[i], quads, &r, &c);
                for (int p = 0; p < g.npass; ++p) {
                    Item it{};
                    // pointer slots are filled per call; offsets go to the side record
                    it.e.d = make_pass_desc(g, p, nullptr, ws[i], hs[i], ws[i], nullptr, c, nullptr, 0, INT_MAX,
                                            base, sign, skip, 0, ra, rb);
                    // quadrants of at most 4 rows (k <= 2) run as direct cells: n x W
                    // items each; the others as tiles
                    it.e.count = g.k <= 2 ? g.n * g.W : it.e.d.n_row_tiles * it.e.d.n_windows;
                    it.e.dep = -1;
                    it.r.img = i;
                    it.r.src_is_ws = p > 0;
                    it.r.src_off = p > 0 ? (int64_t)g.band_byte_off[p - 1] : 0;
                    it.r.dst_is_ws = p + 1 < g.npass;
                    it.r.dst_off = p + 1 < g.npass ? (int64_t)g.band_byte_off[p] : P->out_off[i] * esz;
                    it.p = p;
                    it.G = g.G[p];
                    it.last = p + 1 == g.npass;
                    it.rows = it.e.d.tile_rows;
                    items.push_back(it);
                }
            }
        }
        for (int p = 0; p < 4; ++p)
            for (int G = kMaxG; G >= 0; --G)
                for (int last = 0; last < 2; ++last)
                for (int rows = kTileRows; rows >= kNarrowRows; rows /= 2) {
                    BatchLaunch L{};
                    L.first_group = (int)tmpl.size();
                    int64_t item = 0;
                    for (const Item& it : items) {
                        if (it.p != p || it.G != G || it.last != last || (G > 2 && it.rows != rows)) continue;
                        if (G <= 2 && rows != kTileRows) continue;
                        EngineGroup e = it.e;
                        e.first_item = (int)item;
                        item += e.count;
                        if (item > INT_MAX) {
                            delete P;
                            return fail(FHT_ERR_UNSUPPORTED, "more than 2^31 work items of one kind in one chunk");
                        }
                        tmpl.push_back(e);
                        rel.push_back(it.r);
                    }
                    L.n_groups = (int)tmpl.size() - L.first_group;
                    if (L.n_groups == 0) continue;
                    L.n_items = (int)item;
                    L.G = G;
                    L.rows = rows;
                    L.first = p == 0;
                    L.last = last != 0;
                    P->launches.push_back(L);
                }
        i0 = i1;
    }
    P->n_groups = (int)tmpl.size();
    P->table_bytes = (tmpl.size() * sizeof(EngineGroup) + 255) / 256 * 256;
    // item -> group maps of the tile launches (one load per workgroup instead
    // of a search of the group prefix), unless they would be too large
    std::vector<int32_t> map;
    {
        int64_t total = 0;
        for (const BatchLaunch& L : P->launches)
            if (L.G > 2) total += L.n_items;
        for (BatchLaunch& L : P->launches) L.map_off = -1;
        // FHT_BATCH_MAP=0 in the environment keeps the search (tests of it)
        const char* env = getenv("FHT_BATCH_MAP");
        const bool use_map = !(env && env[0] == '0');
        if (use_map && total <= kBatchMapItems) {
            map.reserve((size_t)total);
            for (BatchLaunch& L : P->launches) {
                if (L.G <= 2) continue;
                L.map_off = (int64_t)map.size();
                for (int g = 0; g < L.n_groups; ++g) {
                    const EngineGroup& e = tmpl[(size_t)L.first_group + g];
                    for (int k = 0; k < e.count; ++k) map.push_back(g);
                }
            }
        }
    }
    // workspace: resolved table, then the bands of the largest chunk
    for (auto& e : tmpl) (void)e;
    for (BatchTemplate& r : rel) {
        if (r.src_is_ws) r.src_off += (int64_t)P->table_bytes;
        if (r.dst_is_ws) r.dst_off += (int64_t)P->table_bytes;
    }
    P->ws_bytes = P->table_bytes + band_peak;

    hipError_t e = hipMalloc((void**)&P->d_tmpl, tmpl.size() * sizeof(EngineGroup));
    if (e == hipSuccess) e = hipMalloc((void**)&P->d_rel, rel.size() * sizeof(BatchTemplate));
    if (e == hipSuccess)
        e = hipMemcpy(P->d_tmpl, tmpl.data(), tmpl.size() * sizeof(EngineGroup), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(P->d_rel, rel.data(), rel.size() * sizeof(BatchTemplate), hipMemcpyHostToDevice);
    if (e == hipSuccess && !map.empty()) e = hipMalloc((void**)&P->d_map, map.size() * sizeof(int32_t));
    if (e == hipSuccess && !map.empty())
        e = hipMemcpy(P->d_map, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(P->d_tmpl);
        hipFree(P->d_rel);
        hipFree(P->d_map);
        delete P;
        return hip_fail(e, "batch plan tables");
    }
    *ws_bytes = P->ws_bytes;
    *out_elems = P->out_elems;
    if (out_offsets)
        for (int i = 0; i < n; ++i) out_offsets[i] = P->out_off[i];
    *plan = P;
    return FHT_OK;
}

static int batch_run(const fht_batch_plan* P, const void* const* imgs, const void* base, int64_t stride, void* hough,
                     void* workspace, size_t ws_bytes, void* stream)
{
    if (!workspace || ws_bytes < P->ws_bytes)
        return fail(FHT_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", P->ws_bytes,
                    workspace ? ws_bytes : 0);
    if ((uintptr_t)workspace & 255) return fail(FHT_ERR_INVALID, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    EngineGroup* table = (EngineGroup*)workspace;
    hipLaunchKernelGGL(fht_batch_fixup_kernel, dim3((P->n_groups + 255) / 256), dim3(256), 0, s, P->d_tmpl, P->d_rel,
                       P->n_groups, imgs, (const unsigned char*)base, stride, (unsigned char*)hough,
                       (unsigned char*)workspace, table);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batch fixup launch");
    const int ti = P->in_t;
    for (const BatchLaunch& L : P->launches) {
        if (L.G <= 2)  // quadrants of at most 4 rows: one thread per Hough cell
            e = launch_table_direct(table + L.first_group, L.n_groups, L.n_items, ti, P->acc_t, s);
        else
            e = launch_table(table + L.first_group, L.n_groups, L.n_items,
                             L.map_off >= 0 ? P->d_map + L.map_off : nullptr, L.G, L.first, L.last, L.rows,
                             L.first ? ti : P->acc_t, P->acc_t, s);
        if (e != hipSuccess) return hip_fail(e, "batch pass launch");
    }
    return FHT_OK;
}

int fht_batch_forward(const fht_batch_plan* P, const void* const* imgs, void* hough, void* workspace, size_t ws_bytes,
                      void* stream)
{
    if (!P || !imgs || !hough) return fail(FHT_ERR_INVALID, "null batch argument");
    return batch_run(P, imgs, nullptr, 0, hough, workspace, ws_bytes, stream);
}

int fht_batch_forward_stack(const fht_batch_plan* P, const void* base, int64_t stride_bytes, void* hough,
                            void* workspace, size_t ws_bytes, void* stream)
{
    if (!P || !base || !hough) return fail(FHT_ERR_INVALID, "null batch argument");
    for (int i = 1; i < P->n; ++i)
        if (P->ws[i] != P->ws[0] || P->hs[i] != P->hs[0])
            return fail(FHT_ERR_INVALID, "a stack needs a plan of equal image sizes");
    const int64_t bytes = (int64_t)P->ws[0] * P->hs[0] * (P->in_t == FHT_U8 ? 1 : 4);
    if (P->n > 1 && stride_bytes < bytes)
        return fail(FHT_ERR_INVALID, "stride %lld bytes < one image (%lld bytes)", (long long)stride_bytes,
                    (long long)bytes);
    return batch_run(P, nullptr, base, stride_bytes, hough, workspace, ws_bytes, stream);
}

int fht_batch_plan_destroy(fht_batch_plan* P)
{
    if (!P) return FHT_OK;
    int dev = 0;
    hipGetDevice(&dev);
    if (dev != P->device) hipSetDevice(P->device);
    hipFree(P->d_tmpl);
    hipFree(P->d_rel);
    hipFree(P->d_map);
    if (dev != P->device) hipSetDevice(dev);
    delete P;
    return FHT_OK;
}

}  // extern "C"
