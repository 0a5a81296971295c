// Per-kernel launch timing with HIP events (see cga_prof_* in cga.h).
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cga_common.h"

namespace cga {
namespace {

struct Rec {
    std::string label;
    hipEvent_t start, stop;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<std::string> g_filter;  // empty: every label
std::vector<Rec> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<double, int64_t>> g_acc;

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

bool wanted(const char *label) {
    if (g_filter.empty()) return true;
    for (const auto &f : g_filter)
        if (f == label) return true;
    return false;
}

// Wait for every pending record and fold it into the totals.
int collect() {
    for (auto &r : g_pending) {
        if (hipEventSynchronize(r.stop) != hipSuccess) return CGA_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return CGA_EHIP;
        auto &a = g_acc[r.label];
        a.first += ms;
        a.second += 1;
        g_pool.push_back(r.start);
        g_pool.push_back(r.stop);
    }
    g_pending.clear();
    return CGA_OK;
}

}  // namespace

ProfScope::ProfScope(const char *label, hipStream_t s) {
    if (!g_on.load(std::memory_order_relaxed)) return;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!wanted(label)) return;
    Rec r{label, take_event(), take_event()};
    if (!r.start || !r.stop) return;
    if (hipEventRecord(r.start, s) != hipSuccess) return;
    stream = s;
    slot = (int)g_pending.size();
    g_pending.push_back(r);
}

ProfScope::~ProfScope() {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(g_pending[slot].stop, stream);
}

}  // namespace cga

using namespace cga;

extern "C" {

int cga_prof_enable(const char *filter) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_filter.clear();
    if (filter && *filter) {
        std::string f(filter);
        size_t p = 0;
        while (p <= f.size()) {
            size_t q = f.find(',', p);
            if (q == std::string::npos) q = f.size();
            if (q > p) g_filter.push_back(f.substr(p, q - p));
            p = q + 1;
        }
    }
    g_on = true;
    return CGA_OK;
}

int cga_prof_disable(void) {
    g_on = false;
    return CGA_OK;
}

int cga_prof_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int st = collect();
    g_acc.clear();
    return st;
}

int cga_prof_read(const char *label, double *total_ms, int64_t *launches) {
    if (!label) return CGA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    CGA_TRY(collect());
    auto it = g_acc.find(label);
    if (total_ms) *total_ms = it == g_acc.end() ? 0.0 : it->second.first;
    if (launches) *launches = it == g_acc.end() ? 0 : it->second.second;
    return CGA_OK;
}

}  // extern "C"
