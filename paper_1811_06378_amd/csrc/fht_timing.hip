// Launch timing (instrumentation, off by default).  While enabled, every
// pass kernel the library enqueues is bracketed by two HIP events recorded
// on the launch stream; fht_timing_report sums the elapsed times per kernel
// instantiation.  Nothing is recorded while the stream is being captured.
// The events are created without the system-scope fence: with it, each
// record wrote back the caches and the forward step of a 4096^2 image took
// about 27 us longer.
#include "fht.h"
#include "fht_internal.h"
#include "fht_plan.h"

#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace fht {
namespace {

constexpr size_t kMaxRecords = size_t(1) << 16;

struct Record {
    int cls;
    int done;  // end event recorded
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::string g_filter;  // record only kernels whose name contains it
int g_device = -1;
std::vector<hipEvent_t> g_events;  // 2 per record: begin, end
std::vector<Record> g_recs;
std::vector<std::string> g_names;
// aggregation (filled by the first report after recording)
bool g_aggregated = false;
std::vector<int64_t> g_launches;
std::vector<double> g_total_ms;

const char* type_name(int t)
{
    switch (t) {
    case 0: return "unsigned char";
    case 1: return "int";
    default: return "float";
    }
}

int class_of(const std::string& name)
{
    for (size_t i = 0; i < g_names.size(); ++i)
        if (g_names[i] == name) return (int)i;
    g_names.push_back(name);
    return (int)g_names.size() - 1;
}

}  // namespace

std::string kernel_name(const char* kernel, int in_t, int acc_t, int GB, bool first, bool last, int op, int nw)
{
    char buf[160];
    char tail[32] = "";
    if (op >= 0 && nw >= 0) snprintf(tail, sizeof tail, ", %d, %d", op, nw);
    else if (op >= 0) snprintf(tail, sizeof tail, ", %d", op);
    else if (nw >= 0) snprintf(tail, sizeof tail, ", %d", nw);
    if (in_t < 0)
        snprintf(buf, sizeof buf, "fht::%s<%s, %d, %s, %s%s>", kernel, type_name(acc_t), GB, first ? "true" : "false",
                 last ? "true" : "false", tail);
    else
        snprintf(buf, sizeof buf, "fht::%s<%s, %s, %d, %s, %s%s>", kernel, type_name(in_t), type_name(acc_t), GB,
                 first ? "true" : "false", last ? "true" : "false", tail);
    return buf;
}

bool timing_on() { return g_on.load(std::memory_order_relaxed); }

int timing_begin(const std::string& name, hipStream_t s)
{
    if (!g_on.load(std::memory_order_relaxed)) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_on.load() || g_recs.size() >= kMaxRecords) return -1;
    if (!g_filter.empty() && name.find(g_filter) == std::string::npos) return -1;
    if (g_device < 0) g_device = dev;
    if (dev != g_device) return -1;
    const size_t slot = g_recs.size();
    while (g_events.size() < 2 * (slot + 1)) {
        // timing-only events: no system-scope fence, which would write back
        // and invalidate the caches at every record and slow the next launch
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
        g_events.push_back(e);
    }
    if (hipEventRecord(g_events[2 * slot], s) != hipSuccess) return -1;
    g_recs.push_back(Record{class_of(name), 0});
    g_aggregated = false;
    return (int)slot;
}

void timing_end(int slot, hipStream_t s)
{
    if (slot < 0) return;
    std::lock_guard<std::mutex> lock(g_mu);
    if ((size_t)slot >= g_recs.size()) return;
    if (hipEventRecord(g_events[2 * (size_t)slot + 1], s) == hipSuccess) g_recs[slot].done = 1;
}

}  // namespace fht

using namespace fht;

extern "C" {

int fht_timing_enable(int on)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (on) {
        g_recs.clear();
        g_names.clear();
        g_launches.clear();
        g_total_ms.clear();
        g_aggregated = false;
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess && dev != g_device) {
            for (hipEvent_t e : g_events) hipEventDestroy(e);
            g_events.clear();
            g_device = dev;
        }
    }
    g_on.store(on != 0);
    return FHT_OK;
}

int fht_timing_filter(const char* substr)
{
    std::lock_guard<std::mutex> lock(g_mu);
    g_filter.assign(substr ? substr : "", substr ? strnlen(substr, 255) : 0);
    return FHT_OK;
}

int fht_timing_report(int index, char* name, int name_cap, int64_t* launches, double* total_ms)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_aggregated) {
        g_launches.assign(g_names.size(), 0);
        g_total_ms.assign(g_names.size(), 0.0);
        for (size_t i = 0; i < g_recs.size(); ++i) {
            if (!g_recs[i].done) continue;
            hipError_t e = hipEventSynchronize(g_events[2 * i + 1]);
            if (e != hipSuccess) return hip_fail(e, "timing event");
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, g_events[2 * i], g_events[2 * i + 1]);
            if (e != hipSuccess) return hip_fail(e, "timing elapsed");
            g_launches[g_recs[i].cls] += 1;
            g_total_ms[g_recs[i].cls] += ms;
        }
        g_aggregated = true;
    }
    if (index < 0 || (size_t)index >= g_names.size())
        return fail(FHT_ERR_INVALID, "timing class %d of %zu", index, g_names.size());
    if (name && name_cap > 0) {
        strncpy(name, g_names[index].c_str(), (size_t)name_cap - 1);
        name[name_cap - 1] = 0;
    }
    if (launches) *launches = g_launches[index];
    if (total_ms) *total_ms = g_total_ms[index];
    return FHT_OK;
}

}  // extern "C"
