// Per-phase kernel timing with HIP events on the caller's stream.
#include <mutex>
#include <vector>

#include "tl_internal.h"
#include "timing.h"

namespace {
// events are reused: creating and destroying them per call costs host time
thread_local std::vector<hipEvent_t> t_events;

hipEvent_t take_event() {
    if (!t_events.empty()) {
        hipEvent_t e = t_events.back();
        t_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

std::mutex g_mu;
bool g_on = false;
double g_ms[TL_NUM_PHASES] = {};
uint64_t g_calls[TL_NUM_PHASES] = {};
}  // namespace

PhaseTimer::PhaseTimer(int phase, hipStream_t s) : phase_(phase), s_(s) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_on) return;
    }
    a_ = take_event();
    b_ = take_event();
    if (!a_ || !b_) return;
    if (hipEventRecord(a_, s_) != hipSuccess) return;
    armed_ = true;
}

void PhaseTimer::stop() {
    if (armed_ && !stopped_) stopped_ = hipEventRecord(b_, s_) == hipSuccess;
}

PhaseTimer::~PhaseTimer() {
    if (armed_) {
        stop();
        float ms = 0.f;
        if (stopped_ && hipEventSynchronize(b_) == hipSuccess && hipEventElapsedTime(&ms, a_, b_) == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_mu);
            g_ms[phase_] += ms;
            g_calls[phase_] += 1;
        }
    }
    if (a_) t_events.push_back(a_);
    if (b_) t_events.push_back(b_);
}

extern "C" {

int tl_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return TL_OK;
}

int tl_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (int i = 0; i < TL_NUM_PHASES; i++) { g_ms[i] = 0; g_calls[i] = 0; }
    return TL_OK;
}

int tl_timing_read(int phase, double *ms, uint64_t *calls) {
    if (phase < 0 || phase >= TL_NUM_PHASES) return TL_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (ms) *ms = g_ms[phase];
    if (calls) *calls = g_calls[phase];
    return TL_OK;
}

}  // extern "C"
