// Event-based kernel timing (see prof.hpp) and its C-ABI accessors.
#include "prof.hpp"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/randrand.h"

namespace rr {

static std::atomic<int> g_on{0};
static std::mutex g_mu;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_pending[PROF_NSLOTS];
static std::vector<float> g_ms[PROF_NSLOTS];

bool prof_enabled() { return g_on.load(std::memory_order_relaxed) != 0; }

void prof_record(int slot, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending[slot].emplace_back(a, b);
}

ProfScope::ProfScope(int slot, hipStream_t st) : slot_(slot), st_(st) {
    if (slot < 0 || !prof_enabled()) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
        a_ = b_ = nullptr;
        return;
    }
    (void)hipEventRecord(a_, st_);
}

ProfScope::~ProfScope() {
    if (!a_) return;
    (void)hipEventRecord(b_, st_);
    prof_record(slot_, a_, b_);
}

static void drain(int slot) {
    for (auto& e : g_pending[slot]) {
        float ms = 0.0f;
        if (hipEventSynchronize(e.second) == hipSuccess &&
            hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
            g_ms[slot].push_back(ms);
        }
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    g_pending[slot].clear();
}

}  // namespace rr

extern "C" {

void rr_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(rr::g_mu);
    for (int s = 0; s < rr::PROF_NSLOTS; ++s) {
        rr::drain(s);
        rr::g_ms[s].clear();
    }
    rr::g_on.store(on ? 1 : 0);
}

rr_status rr_profile_read(int32_t slot, int64_t* count, double* total_ms) {
    if (slot < 0 || slot >= rr::PROF_NSLOTS || !count || !total_ms) return RR_EINVAL;
    std::lock_guard<std::mutex> lk(rr::g_mu);
    rr::drain(slot);
    // launches that a device-side stop flag turned into no-ops (an iteration batch
    // running past convergence) last a few microseconds: count only launches of at
    // least a tenth of the median duration
    std::vector<float> v = rr::g_ms[slot];
    double tot = 0.0;
    int64_t c = 0;
    if (!v.empty()) {
        std::vector<float> srt = v;
        std::nth_element(srt.begin(), srt.begin() + srt.size() / 2, srt.end());
        const float floor_ms = 0.1f * srt[srt.size() / 2];
        for (float x : v)
            if (x >= floor_ms) { tot += x; ++c; }
    }
    *count = c;
    *total_ms = tot;
    return RR_OK;
}

}  // extern "C"
