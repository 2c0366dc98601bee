// Batched forward: placeholder until the persistent kernel lands.
#include "fht.h"
#include "fht_plan.h"

extern "C" {
int fht_batch_plan_create(const int32_t*, const int32_t*, int, unsigned, int, int, fht_batch_plan**, size_t*,
                          int64_t*, int64_t*)
{
    return fht::fail(FHT_ERR_UNSUPPORTED, "batched forward not built yet");
}
int fht_batch_forward(const fht_batch_plan*, const void* const*, void*, void*, size_t, void*)
{
    return fht::fail(FHT_ERR_UNSUPPORTED, "batched forward not built yet");
}
int fht_batch_plan_destroy(fht_batch_plan*) { return FHT_OK; }
}
