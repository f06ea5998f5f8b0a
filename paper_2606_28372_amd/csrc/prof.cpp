// Kernel timing with HIP events recorded on the launch stream around each
// launch (enabled on request; used by the benchmark to time the kernels that
// bound a step against their roofline).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ct_host.h"

namespace {
struct Rec {
    const char* name;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
bool g_suspend = false;
std::string g_only;                 // empty: every kernel
uint32_t g_every = 1;               // record around every g_every-th launch of a name
std::map<std::string, uint64_t> g_seen;   // launches of each name since the last enable
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
unsigned long long* g_boxes = nullptr;   // [4] main boxes, main chunks, fallback boxes, fallback chunks
bool g_count_boxes = false;

hipEvent_t take() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence, whose cache writeback would slow the work that follows
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return e;
}
}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t st) : name_(name), st_(st), a_(nullptr) {
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_on || g_suspend || (!g_only.empty() && g_only != name_)) return;
    if (g_seen[name_]++ % g_every != 0) return;
    a_ = take();
    (void)hipEventRecord((hipEvent_t)a_, st_);
}

ProfScope::~ProfScope() {
    if (!a_) return;
    std::lock_guard<std::mutex> g(g_mu);
    hipEvent_t b = take();
    (void)hipEventRecord(b, st_);
    g_recs.push_back(Rec{name_, (hipEvent_t)a_, b});
}

void prof_suspend(bool on) {
    std::lock_guard<std::mutex> g(g_mu);
    g_suspend = on;
}

unsigned long long* prof_box_counter() {
    std::lock_guard<std::mutex> g(g_mu);
    return g_count_boxes && !g_suspend ? g_boxes : nullptr;
}

extern "C" int ct_prof_count_boxes(int on) {
    std::lock_guard<std::mutex> g(g_mu);
    CT_HIP(hipDeviceSynchronize());
    if (on && !g_boxes) CT_HIP(hipMalloc(&g_boxes, 4 * sizeof(unsigned long long)));
    if (g_boxes) CT_HIP(hipMemset(g_boxes, 0, 4 * sizeof(unsigned long long)));
    g_count_boxes = on != 0;
    return CT_OK;
}

extern "C" int ct_prof_boxes(uint64_t* out4) {
    if (!out4) return ct_fail(CT_EINVAL, "ct_prof_boxes: null argument");
    std::lock_guard<std::mutex> g(g_mu);
    CT_HIP(hipDeviceSynchronize());
    unsigned long long h[4] = {0, 0, 0, 0};
    if (g_boxes) CT_HIP(hipMemcpy(h, g_boxes, sizeof(h), hipMemcpyDeviceToHost));
    for (int k = 0; k < 4; ++k) out4[k] = h[k];
    return CT_OK;
}

extern "C" int ct_prof_enable(int on) {
    std::lock_guard<std::mutex> g(g_mu);
    CT_HIP(hipDeviceSynchronize());
    for (auto& r : g_recs) {
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    g_seen.clear();
    g_on = on != 0;
    return CT_OK;
}

extern "C" int ct_prof_seen(const char* kernel, uint64_t* launches) {
    if (!kernel || !launches) return ct_fail(CT_EINVAL, "ct_prof_seen: null argument");
    std::lock_guard<std::mutex> g(g_mu);
    const auto it = g_seen.find(kernel);
    *launches = it == g_seen.end() ? 0 : it->second;
    return CT_OK;
}

extern "C" int ct_prof_sample(uint32_t every) {
    if (every == 0) return ct_fail(CT_EINVAL, "ct_prof_sample: every must be at least 1");
    std::lock_guard<std::mutex> g(g_mu);
    g_every = every;
    g_seen.clear();
    return CT_OK;
}

extern "C" int ct_prof_select(const char* kernel) {
    std::lock_guard<std::mutex> g(g_mu);
    g_only = kernel ? kernel : "";
    return CT_OK;
}

extern "C" int ct_prof_read(const char* kernel, double* total_ms, uint64_t* launches) {
    if (!kernel || !total_ms || !launches) return ct_fail(CT_EINVAL, "ct_prof_read: null argument");
    std::lock_guard<std::mutex> g(g_mu);
    CT_HIP(hipDeviceSynchronize());
    double t = 0;
    uint64_t n = 0;
    for (auto& r : g_recs) {
        if (std::string(r.name) != kernel) continue;
        float ms = 0;
        CT_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        t += ms;
        n++;
    }
    *total_ms = t;
    *launches = n;
    return CT_OK;
}
