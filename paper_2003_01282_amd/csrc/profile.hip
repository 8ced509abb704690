// Optional kernel timing with HIP events.  When enabled, the library brackets
// each launch of its stage kernels with a pair of events on the launch stream;
// slaq_profile_read waits for them and sums the elapsed times per kernel name.
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "profile.hpp"

namespace slaq {

namespace {
struct Record {
    const char* name;
    hipEvent_t start, stop;
};
std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Record> g_records;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

int prof_begin(const char* name, hipStream_t st) {
    if (!g_on.load(std::memory_order_relaxed)) return -1;
    // launches being captured into a hipGraph are not timed: an event
    // recorded during capture becomes a graph node, not a timestamp
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    Record r{name, take_event(), take_event()};
    if (!r.start || !r.stop) return -1;
    if (hipEventRecord(r.start, st) != hipSuccess) return -1;
    g_records.push_back(r);
    return (int)g_records.size() - 1;
}

void prof_end(int token, hipStream_t st) {
    if (token < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((size_t)token < g_records.size()) (void)hipEventRecord(g_records[token].stop, st);
}

}  // namespace slaq

using namespace slaq;

extern "C" {

slaq_status slaq_profile_enable(int on) {
    g_on.store(on != 0);
    return SLAQ_OK;
}

slaq_status slaq_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& r : g_records) {
        (void)hipEventSynchronize(r.stop);
        g_pool.push_back(r.start);
        g_pool.push_back(r.stop);
    }
    g_records.clear();
    return SLAQ_OK;
}

slaq_status slaq_profile_read(const char* kernel, int64_t* launches, double* total_ms) {
    clear_error();
    SLAQ_REQUIRE(kernel && launches && total_ms, SLAQ_ERR_INVALID_ARG, "NULL pointer argument");
    std::lock_guard<std::mutex> lk(g_mu);
    int64_t cnt = 0;
    double ms = 0.0;
    for (auto& r : g_records) {
        if (std::strcmp(r.name, kernel) != 0) continue;
        SLAQ_HIP(hipEventSynchronize(r.stop));
        float t = 0.0f;
        SLAQ_HIP(hipEventElapsedTime(&t, r.start, r.stop));
        ms += t;
        ++cnt;
    }
    *launches = cnt;
    *total_ms = ms;
    return SLAQ_OK;
}

}  // extern "C"
