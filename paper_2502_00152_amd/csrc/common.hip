// Error reporting, device scratch and launch timing for libhisq.
#include <mutex>

#include "hisq_internal.h"

namespace hisq {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

hisq_status fail(hisq_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

// ---------------------------------------------------------------- workspace
Workspace::~Workspace() { release(); }

void Workspace::release() {
    for (auto &kv : bufs_)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    bufs_.clear();
}

hisq_status Workspace::get(const char *name, size_t bytes, void **ptr) {
    Buf &b = bufs_[name];
    if (b.bytes < bytes) {
        if (b.ptr) {
            HISQ_HIP(hipDeviceSynchronize());
            HISQ_HIP(hipFree(b.ptr));
            b.ptr = nullptr;
            b.bytes = 0;
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess)
            return fail(HISQ_ERR_OOM, std::string("scratch '") + name + "' of " +
                                          std::to_string(bytes) + " bytes: " +
                                          hipGetErrorString(e));
        // arrival counters and partial sums start from zero
        HISQ_HIP(hipMemset(p, 0, bytes));
        b.ptr = p;
        b.bytes = bytes;
    }
    *ptr = b.ptr;
    return HISQ_OK;
}

// ---------------------------------------------------------------- profiling
namespace {
struct ProfRecord {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pairs;
    int64_t seen = 0;  // launches of the class since profiling was enabled
};
std::mutex g_prof_mu;
bool g_prof_on = false;
int g_prof_period = 1;  // time every g_prof_period-th launch of each class
std::map<std::string, ProfRecord> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

ProfileScope::ProfileScope(const char *cls, hipStream_t s) : s_(s), cls_(cls) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    auto &rec = g_prof[cls];
    if (rec.seen++ % g_prof_period != 0) return;
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b) return;
    rec.pairs.emplace_back(a, b);
    slot_ = (int)rec.pairs.size() - 1;
    (void)hipEventRecord(a, s);
}

ProfileScope::~ProfileScope() {
    if (slot_ < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    (void)hipEventRecord(g_prof[cls_].pairs[slot_].second, s_);
}

}  // namespace hisq

using namespace hisq;

extern "C" {

const char *hisq_last_error(void) { return g_last_error.c_str(); }

int hisq_abi_version(void) { return HISQ_ABI_VERSION; }

hisq_status hisq_set_tuning(const char *key, int64_t value) {
    if (!key) return fail(HISQ_ERR_INVALID_ARG, "hisq_set_tuning: null key");
    return dslash_set_tuning(key, value);
}

hisq_status hisq_profile_enable(int on) {
    if (on < 0) return fail(HISQ_ERR_INVALID_ARG, "hisq_profile_enable: period must be >= 0");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    g_prof_period = on > 0 ? on : 1;
    for (auto &kv : g_prof) kv.second.seen = 0;
    return HISQ_OK;
}

hisq_status hisq_profile_read(const char *kernel_class, int64_t *launches, double *total_ms) {
    if (!kernel_class || !launches || !total_ms)
        return fail(HISQ_ERR_INVALID_ARG, "hisq_profile_read: null argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    *launches = 0;
    *total_ms = 0.0;
    auto it = g_prof.find(kernel_class);
    if (it == g_prof.end()) return HISQ_OK;
    for (auto &pr : it->second.pairs) {
        HISQ_HIP(hipEventSynchronize(pr.second));
        float ms = 0.f;
        HISQ_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        *total_ms += ms;
        *launches += 1;
        g_event_pool.push_back(pr.first);
        g_event_pool.push_back(pr.second);
    }
    it->second.pairs.clear();
    return HISQ_OK;
}

}  // extern "C"
