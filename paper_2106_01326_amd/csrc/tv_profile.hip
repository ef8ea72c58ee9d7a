// Per-stage HIP-event timing: events come from a reusable pool; a record
// holds (stage, start, end) until tv_profile_read sums and releases it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "tv.h"
#include "tv_profile.h"

namespace tv {
namespace {

struct Record {
    int stage;
    hipEvent_t start, end;
};

std::mutex g_mu;
bool g_on = false;
int64_t g_calls = 0;
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

const char *kNames[kStageCount] = {"clear", "ingest", "bin", "voxelize", "large"};

}  // namespace

bool profile_on() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_on;
}

void profile_count_call() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_on) ++g_calls;
}

StageScope::StageScope(int stage, hipStream_t s) : stage_(stage), s_(s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    start_ = take_event();
    if (start_ && hipEventRecord(start_, s_) != hipSuccess) {
        g_pool.push_back(start_);
        start_ = nullptr;
    }
}

StageScope::~StageScope() {
    if (!start_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t end = take_event();
    if (!end || hipEventRecord(end, s_) != hipSuccess) {
        g_pool.push_back(start_);
        if (end) g_pool.push_back(end);
        return;
    }
    g_records.push_back({stage_, start_, end});
}

}  // namespace tv

extern "C" {

tv_status tv_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(tv::g_mu);
    tv::g_on = on != 0;
    return TV_OK;
}

tv_status tv_profile_read(double *ms_out, int32_t max_stages, int32_t *n_stages, int64_t *n_calls) {
    if (!ms_out || max_stages < 0) return TV_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(tv::g_mu);
    for (int i = 0; i < max_stages; ++i) ms_out[i] = 0.0;
    tv_status st = TV_OK;
    for (const tv::Record &r : tv::g_records) {
        float ms = 0.f;
        if (hipEventSynchronize(r.end) != hipSuccess ||
            hipEventElapsedTime(&ms, r.start, r.end) != hipSuccess)
            st = TV_ERR_HIP;
        if (r.stage < max_stages) ms_out[r.stage] += ms;
        tv::g_pool.push_back(r.start);
        tv::g_pool.push_back(r.end);
    }
    tv::g_records.clear();
    if (n_stages) *n_stages = tv::kStageCount;
    if (n_calls) *n_calls = tv::g_calls;
    tv::g_calls = 0;
    return st;
}

const char *tv_profile_stage_name(int32_t stage) {
    if (stage < 0 || stage >= tv::kStageCount) return "unknown";
    return tv::kNames[stage];
}

}  // extern "C"
