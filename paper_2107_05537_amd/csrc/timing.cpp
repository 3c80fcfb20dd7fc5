// Opt-in per-stage timing of pmlsh_ann: for each enabled stage, the stage's
// kernel launches are bracketed by two HIP events on the caller's stream. The
// events are resolved (synchronised and summed) only when the totals are
// read, and then reused, so a timed stage adds two event records per launch
// and no host synchronisation to the query path.

#include <atomic>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace pmlsh {
namespace {

struct Pending {
    int stage;
    hipEvent_t a, b;
};

std::mutex g_mu;
unsigned g_mask = 0;                 // stages being timed (bit s = stage s)
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_free;      // resolved events, reused
double g_ms[PMLSH_N_STAGES] = {0};
int64_t g_count[PMLSH_N_STAGES] = {0};

}  // namespace

bool timing_enabled(int stage) {
    std::lock_guard<std::mutex> lk(g_mu);
    return (g_mask >> stage) & 1u;
}

void timing_set(unsigned mask) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_mask = mask;
}

namespace {
hipEvent_t take_event() {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_free.empty()) {
            hipEvent_t e = g_free.back();
            g_free.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    PMLSH_HIP(hipEventCreate(&e));
    return e;
}
}  // namespace

namespace {
thread_local bool g_off = false;   // set by TimingOff on this thread
}  // namespace

TimingOff::TimingOff() : prev_(g_off) { g_off = true; }
TimingOff::~TimingOff() { g_off = prev_; }

StageTimer::StageTimer(int stage, hipStream_t st) : stage_(stage), st_(st) {
    if (g_off || !timing_enabled(stage)) return;
    a_ = take_event();
    b_ = take_event();
    PMLSH_HIP(hipEventRecord(a_, st_));
    on_ = true;
}

StageTimer::~StageTimer() {
    if (!on_) return;
    if (hipEventRecord(b_, st_) != hipSuccess) {
        (void)hipEventDestroy(a_);
        (void)hipEventDestroy(b_);
        return;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({stage_, a_, b_});
}

void timing_read(pmlsh_ann_timing* out, bool reset) {
    std::vector<Pending> p;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        p.swap(g_pending);
    }
    for (const Pending& e : p) {
        float ms = 0.f;
        if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_mu);
            g_ms[e.stage] += ms;
            g_count[e.stage] += 1;
        }
        std::lock_guard<std::mutex> lk(g_mu);
        g_free.push_back(e.a);
        g_free.push_back(e.b);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (int i = 0; i < PMLSH_N_STAGES; ++i) {
        out->ms[i] = g_ms[i];
        out->launches[i] = g_count[i];
        if (reset) { g_ms[i] = 0; g_count[i] = 0; }
    }
}

// ---------------------------------------------------------------- switches
namespace {
std::atomic<int64_t> g_tune[PMLSH_N_TUNE] = {{2048}, {1}, {0}, {0}, {0}};
}  // namespace

int64_t tune_default(int key) {
    return key == PMLSH_TUNE_GROUP_LIST ? 2048
           : key == PMLSH_TUNE_FP32_PATH || key == PMLSH_TUNE_ACP_FIRST_CAP ||
                   key == PMLSH_TUNE_SCAN_SHAPE
               ? 0
               : 1;
}
int64_t tune_get(int key) { return g_tune[key].load(std::memory_order_relaxed); }
void tune_set(int key, int64_t value) { g_tune[key].store(value, std::memory_order_relaxed); }

}  // namespace pmlsh
