// Kernel timing with HIP events recorded on the launch stream.  Each
// instrumented launch records a start and a stop event; om_profile_query
// waits for the recorded events and sums the elapsed times per kernel class.
#include "profile.hpp"

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace omss {

namespace {
struct Cls {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    int64_t launches = 0;
    double bytes = 0.0;
    double ms = 0.0;
};
std::mutex g_mu;
bool g_on = false;
std::map<std::string, Cls> g_cls;
std::vector<hipEvent_t> g_pool;

hipEvent_t take() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drain(Cls& c) {
    for (auto& pr : c.pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess)
            c.ms += ms;
        g_pool.push_back(pr.first);
        g_pool.push_back(pr.second);
    }
    c.pending.clear();
}
}  // namespace

bool profile_enabled() { return g_on; }

ProfScope::ProfScope(const char* cls, hipStream_t s, double bytes) : cls_(cls), s_(s), bytes_(bytes) {
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    a_ = take();
    b_ = take();
    if (a_) (void)hipEventRecord(a_, s_);
}

void ProfScope::stop() {
    if (!a_ || !b_ || stopped_) return;
    (void)hipEventRecord(b_, s_);
    stopped_ = true;
}

ProfScope::~ProfScope() {
    if (!a_ || !b_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!stopped_) (void)hipEventRecord(b_, s_);
    Cls& c = g_cls[cls_];
    c.pending.emplace_back(a_, b_);
    c.launches += 1;
    c.bytes += bytes_;
}

}  // namespace omss

using namespace omss;

extern "C" {

void om_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
}

void om_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_cls) drain(kv.second);
    g_cls.clear();
}

om_status om_profile_query(const char* kernel_class, int64_t* launches, double* total_ms, double* bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!kernel_class) { set_error("null kernel class"); return OM_EINVAL; }
    auto it = g_cls.find(kernel_class);
    if (it == g_cls.end()) {
        if (launches) *launches = 0;
        if (total_ms) *total_ms = 0.0;
        if (bytes) *bytes = 0.0;
        return OM_OK;
    }
    drain(it->second);
    if (launches) *launches = it->second.launches;
    if (total_ms) *total_ms = it->second.ms;
    if (bytes) *bytes = it->second.bytes;
    return OM_OK;
}

}  // extern "C"
