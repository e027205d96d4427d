// timing.hip -- optional per-kernel timing of the brick-binned operator
// kernels with HIP events recorded on the launch stream (measurement support;
// off by default, no effect on results).
#include <atomic>
#include <mutex>
#include <utility>
#include <vector>

#include "csg_internal.h"

namespace csg {
namespace {

constexpr size_t kMaxPending = 8192;  // recorded launches per kernel between reads

std::mutex g_mu;
std::atomic<int> g_enabled{0};
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_pending[kTimedKernels];
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence (cache write-back and invalidate)
    // when the event is recorded, which would stall and cool the next launch
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

void timing_set(int on) { g_enabled.store(on ? 1 : 0); }

hipEvent_t timing_begin(int kernel, hipStream_t st) {
    if (!g_enabled.load() || kernel < 0 || kernel >= kTimedKernels) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_pending[kernel].size() >= kMaxPending) return nullptr;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, st) != hipSuccess) {
        g_pool.push_back(e);
        return nullptr;
    }
    return e;
}

void timing_end(int kernel, hipEvent_t start, hipStream_t st) {
    if (!start) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t e = take_event();
    if (!e || hipEventRecord(e, st) != hipSuccess) {
        if (e) g_pool.push_back(e);
        g_pool.push_back(start);
        return;
    }
    g_pending[kernel].emplace_back(start, e);
}

hipError_t timing_read(int kernel, double *total_ms, int64_t *launches) {
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0;
    int64_t cnt = 0;
    hipError_t err = hipSuccess;
    for (auto &pr : g_pending[kernel]) {
        if (err == hipSuccess) {
            err = hipEventSynchronize(pr.second);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, pr.first, pr.second);
            if (err == hipSuccess) {
                tot += ms;
                ++cnt;
            }
        }
        g_pool.push_back(pr.first);
        g_pool.push_back(pr.second);
    }
    g_pending[kernel].clear();
    *total_ms = tot;
    *launches = cnt;
    return err;
}

}  // namespace csg
