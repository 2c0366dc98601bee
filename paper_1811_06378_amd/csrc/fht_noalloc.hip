// Allocation-free forward transform: fht_forward with its scratch (the
// intermediate bands of the passes, plus the persistent engine's counters)
// held in a file-scope device array instead of a caller workspace, for
// callers that cannot allocate device memory.
//
// The array is a symbol of the library's code object, so every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// names a host-side stand-in, not device memory): its device address is
// looked up once per device with hipGetSymbolAddress and only that address
// is used.

#include "fht.h"
#include "fht_internal.h"
#include "fht_plan.h"

#include <mutex>

namespace fht {

static __device__ __align__(256) unsigned char scratch[FHT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices];

// Device address of `scratch` on the current device, looked up on the first
// call for that device (with that device current) and kept.
static int scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(FHT_ERR_UNSUPPORTED, "device %d: the allocation-free forward supports devices 0..%d", dev,
                    kMaxScratchDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || ((uintptr_t)ptr & 255)) return fail(FHT_ERR_HIP, "scratch symbol has no aligned device address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FHT_OK;
}

}  // namespace fht

using namespace fht;

extern "C" int fht_forward_noalloc(const void* img, int in_t, int w, int h, int64_t ld_img, void* hough, int acc_t,
                                   int64_t ld_hough, unsigned quads, unsigned flags, void* stream)
{
    size_t need = 0;
    int rc = forward_check(img, in_t, w, h, ld_img, hough, acc_t, ld_hough, quads, flags, &need);
    if (rc) return rc;
    if (need > (size_t)FHT_NOALLOC_SCRATCH_BYTES)
        return fail(FHT_ERR_UNSUPPORTED,
                    "this transform needs %zu bytes of scratch; the allocation-free forward holds %zu (use "
                    "fht_forward with a workspace)",
                    need, (size_t)FHT_NOALLOC_SCRATCH_BYTES);
    void* ptr = nullptr;
    rc = scratch_address(&ptr);
    if (rc) return rc;
    return fht_forward(img, in_t, w, h, ld_img, hough, acc_t, ld_hough, quads, flags, ptr,
                       (size_t)FHT_NOALLOC_SCRATCH_BYTES, stream);
}
