// Per-kernel timing with HIP events recorded on the launching stream.
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace rt {
namespace {

struct Rec {
    const char *name;
    hipEvent_t a, b;
};

std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Rec> g_recs;

}  // namespace

KTimer::KTimer(const char *name, hipStream_t s) : name_(name), s_(s)
{
    if (!g_on.load(std::memory_order_relaxed)) return;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) return;
    if (hipEventRecord(a_, s_) == hipSuccess) live_ = true;
}

void KTimer::stop()
{
    if (!live_) return;
    live_ = false;
    if (hipEventRecord(b_, s_) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back({name_, a_, b_});
}

KTimer::~KTimer() { stop(); }

}  // namespace rt

using namespace rt;

extern "C" int rt_timing_enable(int on)
{
    g_on.store(on ? 1 : 0);
    return RT_OK;
}

extern "C" int rt_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (Rec &r : g_recs) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_recs.clear();
    return RT_OK;
}

extern "C" int rt_timing_read(const char *kernel, double *total_ms, int64_t *launches)
{
    if (!kernel || !total_ms || !launches) return fail(RT_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0;
    int64_t n = 0;
    for (Rec &r : g_recs) {
        if (std::strcmp(r.name, kernel) != 0) continue;
        RT_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        RT_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return RT_OK;
}
