// apply_H launch timing with HIP events recorded on the launch stream.
#include "timing.hpp"

#include <mutex>
#include <utility>
#include <vector>

#include "common.hpp"

namespace syk {

namespace {
std::mutex g_mu;
bool g_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;   // completed begin/end pairs
hipEvent_t g_open = nullptr;                                // begin without end yet
}  // namespace

void timing_enable(bool on)
{
    std::lock_guard<std::mutex> l(g_mu);
    g_on = on;
}

bool timing_enabled()
{
    std::lock_guard<std::mutex> l(g_mu);
    return g_on;
}

void timing_begin(hipStream_t s)
{
    std::lock_guard<std::mutex> l(g_mu);
    if (!g_on) return;
    hipEvent_t e;
    SYK_HIP(hipEventCreate(&e));
    SYK_HIP(hipEventRecord(e, s));
    g_open = e;
}

void timing_end(hipStream_t s)
{
    std::lock_guard<std::mutex> l(g_mu);
    if (!g_on || !g_open) return;
    hipEvent_t e;
    SYK_HIP(hipEventCreate(&e));
    SYK_HIP(hipEventRecord(e, s));
    g_events.emplace_back(g_open, e);
    g_open = nullptr;
}

void timing_read(int64_t* launches, double* total_ms)
{
    std::lock_guard<std::mutex> l(g_mu);
    double tot = 0.0;
    for (auto& p : g_events) {
        SYK_HIP(hipEventSynchronize(p.second));
        float ms = 0.f;
        SYK_HIP(hipEventElapsedTime(&ms, p.first, p.second));
        tot += ms;
    }
    if (launches) *launches = (int64_t)g_events.size();
    if (total_ms) *total_ms = tot;
}

void timing_reset()
{
    std::lock_guard<std::mutex> l(g_mu);
    for (auto& p : g_events) {
        (void)hipEventSynchronize(p.second);
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    g_events.clear();
    if (g_open) (void)hipEventDestroy(g_open);
    g_open = nullptr;
}

}  // namespace syk
