// ktimer.cpp -- live kernel timing for measurement (deinsum_kernel_timing): while on,
// the main kernel of every MTTKRP / TTMc call is bracketed by two HIP events on the
// stream it is launched on, so a benchmark can read that kernel's own duration (the
// small set-up and reduction kernels of the call excluded) without a profiler.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.h"

namespace deinsum {

namespace {

struct Slot {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Slot> g_slots;  // events created at enable
size_t g_used = 0;

void release_all()
{
    for (Slot &s : g_slots) {
        if (s.a) (void)hipEventDestroy(s.a);
        if (s.b) (void)hipEventDestroy(s.b);
    }
    g_slots.clear();
    g_used = 0;
}

}  // namespace

int ktimer_begin(void *stream, int kind)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || g_used >= g_slots.size()) return -1;
    const int idx = static_cast<int>(g_used++);
    g_slots[idx].kind = kind;
    (void)hipEventRecord(g_slots[idx].a, s);
    return idx;
}

void ktimer_end(int idx, void *stream)
{
    if (idx < 0) return;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    if (static_cast<size_t>(idx) < g_slots.size()) (void)hipEventRecord(g_slots[idx].b, s);
}

}  // namespace deinsum

using namespace deinsum;

extern "C" {

deinsum_status deinsum_kernel_timing(int32_t enable, int64_t capacity)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!enable) {
        g_on = false;
        return DEINSUM_OK;
    }
    if (capacity < 1 || capacity > (int64_t(1) << 20))
        return fail(DEINSUM_ERR_INVALID_ARG, "kernel_timing: capacity must be 1..2^20");
    (void)hipDeviceSynchronize();  // earlier records may still be pending
    release_all();
    g_slots.resize(static_cast<size_t>(capacity));
    for (Slot &s : g_slots)
        if (hipEventCreate(&s.a) != hipSuccess || hipEventCreate(&s.b) != hipSuccess) {
            (void)hipGetLastError();
            release_all();
            return fail(DEINSUM_ERR_DEVICE, "kernel_timing: event creation failed");
        }
    g_on = true;
    return DEINSUM_OK;
}

deinsum_status deinsum_kernel_times(int64_t max_n, int32_t *kind, double *ms, int64_t *n)
{
    if (!n || max_n < 0 || (max_n > 0 && (!kind || !ms)))
        return fail(DEINSUM_ERR_INVALID_ARG, "kernel_times: bad argument");
    std::lock_guard<std::mutex> lk(g_mu);
    const int64_t cnt = std::min<int64_t>(max_n, static_cast<int64_t>(g_used));
    for (int64_t i = 0; i < cnt; ++i) {
        Slot &s = g_slots[static_cast<size_t>(i)];
        float t = 0;
        if (hipEventSynchronize(s.b) != hipSuccess || hipEventElapsedTime(&t, s.a, s.b) != hipSuccess) {
            (void)hipGetLastError();
            return fail(DEINSUM_ERR_DEVICE, "kernel_times: event read failed");
        }
        kind[i] = s.kind;
        ms[i] = t;
    }
    *n = cnt;
    g_used = 0;
    return DEINSUM_OK;
}

}  // extern "C"
