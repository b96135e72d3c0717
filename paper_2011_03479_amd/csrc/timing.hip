// Kernel timing for measurement (gempe_timing_enable / gempe_timing_read).
//
// While timing is on, the launchers bracket the launches of each kernel class with a pair
// of HIP events recorded on the launch's own stream, so the elapsed time between them is
// the device time of those launches (plus nothing else on that stream).  Brackets are
// closed on the host thread that opened them; completed pairs are kept under a mutex
// until gempe_timing_read waits for them and sums them.  With timing off a bracket costs
// one relaxed atomic load.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "internal.h"

namespace {

struct Pair {
    hipEvent_t start, stop;
    int launches;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Pair> g_done[kTkClasses];
std::vector<hipEvent_t> g_pool;  // events of read pairs, reused

thread_local std::vector<std::pair<int, hipEvent_t>> t_open;  // (class, start) of open brackets

hipEvent_t take_event() {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_pool.empty()) {
            hipEvent_t e = g_pool.back();
            g_pool.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

}  // namespace

bool gempe_timing_on() { return g_on.load(std::memory_order_relaxed); }

void gempe_timing_begin(int cls, hipStream_t s) {
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) != hipSuccess) {
        (void)hipGetLastError();
        e = nullptr;
    }
    t_open.emplace_back(cls, e);
}

void gempe_timing_end(int cls, hipStream_t s, int launches) {
    if (t_open.empty()) return;
    const std::pair<int, hipEvent_t> o = t_open.back();
    t_open.pop_back();
    if (!o.second || o.first != cls) return;
    hipEvent_t e = take_event();
    if (!e) return;
    if (hipEventRecord(e, s) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_done[cls].push_back(Pair{o.second, e, launches});
}

extern "C" gempe_status gempe_timing_enable(int32_t on) {
    g_on.store(on != 0, std::memory_order_relaxed);
    return GEMPE_OK;
}

extern "C" gempe_status gempe_timing_read(int32_t kclass, int64_t *launches, double *total_ms) {
    if (kclass < 0 || kclass >= kTkClasses) return gempe_fail(GEMPE_ERR_ARG, "timing_read: unknown kernel class");
    if (!launches || !total_ms) return gempe_fail(GEMPE_ERR_ARG, "timing_read: null output");
    std::vector<Pair> pairs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        pairs.swap(g_done[kclass]);
    }
    int64_t nl = 0;
    double ms = 0.0;
    gempe_status st = GEMPE_OK;
    for (const Pair &p : pairs) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(p.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, p.start, p.stop);
        if (e != hipSuccess && st == GEMPE_OK)
            st = gempe_fail(GEMPE_ERR_HIP, std::string("timing_read: ") + hipGetErrorString(e));
        nl += p.launches;
        ms += (double)t;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const Pair &p : pairs) {
            g_pool.push_back(p.start);
            g_pool.push_back(p.stop);
        }
    }
    *launches = nl;
    *total_ms = ms;
    return st;
}
