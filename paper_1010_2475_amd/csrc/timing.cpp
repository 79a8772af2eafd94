// Optional per-kernel timing: events stamped at the start and end of the timed
// kernel by the runtime (hipExtLaunchKernel), on the kernel's own stream.
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "api_internal.hpp"

namespace mmvm {

namespace {
struct Pending {
    std::string name;
    hipEvent_t a, b;
};
struct Acc {
    double ms = 0.0;
    int64_t n = 0;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, Acc> g_acc;

hipEvent_t get_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void collect_locked()
{
    for (auto& p : g_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            Acc& a = g_acc[p.name];
            a.ms += ms;
            a.n += 1;
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}
}  // namespace

namespace {
std::atomic<int64_t> g_graph_replays{0};
}

void count_graph_replays(int64_t n) { g_graph_replays += n; }
int64_t graph_replays() { return g_graph_replays.load(); }

TimingSlot*& timing_slot()
{
    static thread_local TimingSlot* slot = nullptr;
    return slot;
}

bool timing_on()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_on;
}

void* timing_begin(hipStream_t st)
{
    (void)st;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return nullptr;
    TimingSlot* ts = new TimingSlot();
    ts->start = get_event();
    ts->stop = get_event();
    timing_slot() = ts;
    return ts;
}

void timing_end(void* tok, const char* name, hipStream_t st)
{
    (void)st;
    if (!tok) return;
    TimingSlot* ts = (TimingSlot*)tok;
    timing_slot() = nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (ts->used) {
        g_pending.push_back(Pending{name, ts->start, ts->stop});
        if (g_pending.size() > 4096) collect_locked();
    } else {
        g_pool.push_back(ts->start);
        g_pool.push_back(ts->stop);
    }
    delete ts;
}

}  // namespace mmvm

using namespace mmvm;

extern "C" {

mmvm_status mmvm_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    collect_locked();
    g_on = on != 0;
    if (on) g_acc.clear();
    return MMVM_OK;
}

mmvm_status mmvm_timing_get(const char* kernel, double* total_ms, int64_t* launches)
{
    if (!kernel || !total_ms || !launches) return MMVM_EINVAL;
    if (std::string(kernel) == "graph") {  // replays of captured stepping graphs (counted always)
        *total_ms = 0.0;
        *launches = graph_replays();
        return MMVM_OK;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    collect_locked();
    auto it = g_acc.find(kernel);
    if (it == g_acc.end()) {
        *total_ms = 0.0;
        *launches = 0;
        return MMVM_ENOTFOUND;
    }
    *total_ms = it->second.ms;
    *launches = it->second.n;
    return MMVM_OK;
}
}
