// Error reporting, device scratch and launch timing for libhisq.
#include <mutex>

#include <algorithm>

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

void Workspace::release_one(const char *name) {
    auto it = bufs_.find(name);
    if (it == bufs_.end()) return;
    if (it->second.ptr) (void)hipFree(it->second.ptr);
    bufs_.erase(it);
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
        // No kernel reads scratch it has not written in the same solve (the
        // reductions store every partial before a later kernel sums them, and
        // the CG state is set by its init kernel), so the contents of a new
        // buffer do not matter.  It is still cleared, and the clear completed
        // before the buffer is handed out (the solvers' non-blocking streams
        // do not wait for the null stream), so that a stray read of it is
        // reproducible.
        HISQ_HIP(hipMemset(p, 0, bytes));
        HISQ_HIP(hipDeviceSynchronize());
        b.ptr = p;
        b.bytes = bytes;
    }
    *ptr = b.ptr;
    return HISQ_OK;
}

// ------------------------------------------------------------ solver stream
GraphChunk::~GraphChunk() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
}

// ------------------------------------------------------ combined chunks
thread_local ChunkGroup *t_chunk_group = nullptr;
thread_local int t_chunk_sys = -1;

ChunkGroup::~ChunkGroup() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    for (hipEvent_t e : events_) (void)hipEventDestroy(e);
    if (origin_) (void)hipStreamDestroy(origin_);
}

hisq_status ChunkGroup::run(hipStream_t s, int sys, const std::function<hisq_status()> &body) {
    std::unique_lock<std::mutex> lk(mu_);
    if (round_status_ != HISQ_OK) return fail(round_status_, round_error_);
    const uint64_t mine = round_;
    pending_.push_back(Pending{s, sys, &body});
    if ((int)pending_.size() == active_) launch_locked();
    else cv_.wait(lk, [&] { return round_ != mine; });
    if (round_status_ != HISQ_OK) return fail(round_status_, round_error_);
    return HISQ_OK;
}

void ChunkGroup::leave() {
    std::lock_guard<std::mutex> lk(mu_);
    --active_;
    if (active_ > 0 && (int)pending_.size() == active_) launch_locked();
}

// Capture the pending chunks into graph_/exec_ (members in system order).
hisq_status ChunkGroup::capture_locked() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    exec_ = nullptr;
    graph_ = nullptr;
    const size_t n = pending_.size();
    while (events_.size() < n + 1) {
        hipEvent_t e = nullptr;
        HISQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        events_.push_back(e);
    }
    HISQ_HIP(hipStreamBeginCapture(origin_, hipStreamCaptureModeRelaxed));
    hisq_status st = HISQ_OK;
    hipError_t e = hipEventRecord(events_[n], origin_);  // the fork
    for (size_t i = 0; i < n && e == hipSuccess && st == HISQ_OK; ++i) {
        e = hipStreamWaitEvent(pending_[i].s, events_[n], 0);
        if (e != hipSuccess) break;
        st = (*pending_[i].body)();
        if (st != HISQ_OK) break;
        e = hipEventRecord(events_[i], pending_[i].s);  // the join
        if (e == hipSuccess) e = hipStreamWaitEvent(origin_, events_[i], 0);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(origin_, &graph);
    if (st != HISQ_OK || e != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (st != HISQ_OK) return st;
        HISQ_HIP(e != hipSuccess ? e : ee);
    }
    graph_ = graph;
    HISQ_HIP(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
    return HISQ_OK;
}

void ChunkGroup::launch_locked() {
    std::sort(pending_.begin(), pending_.end(),
              [](const Pending &a, const Pending &b) { return a.sys < b.sys; });
    std::vector<std::pair<hipStream_t, int>> key;
    for (const Pending &p : pending_) key.emplace_back(p.s, p.sys);
    hisq_status st = HISQ_OK;
    auto check = [&](hipError_t e, const char *what) {
        if (st == HISQ_OK && e != hipSuccess)
            st = fail(HISQ_ERR_HIP, std::string("chunk group: ") + what + ": " +
                                        hipGetErrorString(e));
    };
    if (!origin_) check(hipStreamCreateWithFlags(&origin_, hipStreamNonBlocking), "stream");
    if (st == HISQ_OK && (key != key_ || !exec_)) {
        st = capture_locked();
        key_ = st == HISQ_OK ? key : std::vector<std::pair<hipStream_t, int>>();
    }
    // the graph runs after every member's earlier work, and every member's
    // later work after the graph
    const size_t n = pending_.size();
    for (size_t i = 0; i < n && st == HISQ_OK; ++i) {
        check(hipEventRecord(events_[i], pending_[i].s), "record");
        check(hipStreamWaitEvent(origin_, events_[i], 0), "wait");
    }
    if (st == HISQ_OK) check(hipGraphLaunch(exec_, origin_), "graph launch");
    if (st == HISQ_OK) check(hipEventRecord(events_[n], origin_), "record");
    for (size_t i = 0; i < n && st == HISQ_OK; ++i)
        check(hipStreamWaitEvent(pending_[i].s, events_[n], 0), "wait");
    if (st != HISQ_OK) {
        round_status_ = st;
        round_error_ = hisq_last_error();
    }
    pending_.clear();
    ++round_;
    cv_.notify_all();
}

hisq_status solver_stream(hisq_gauge_s *g, hipStream_t caller, hipStream_t *out) {
    if (!g->cg_stream) HISQ_HIP(hipStreamCreateWithFlags(&g->cg_stream, hipStreamNonBlocking));
    hipEvent_t e = nullptr;
    HISQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipError_t r = hipEventRecord(e, caller);
    if (r == hipSuccess) r = hipStreamWaitEvent(g->cg_stream, e, 0);
    (void)hipEventDestroy(e);  // released once the wait is resolved
    HISQ_HIP(r);
    *out = g->cg_stream;
    return HISQ_OK;
}

hisq_status solver_stream_done(hisq_gauge_s *g, hipStream_t caller) {
    hipEvent_t e = nullptr;
    HISQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipError_t r = hipEventRecord(e, g->cg_stream);
    if (r == hipSuccess) r = hipStreamWaitEvent(caller, e, 0);
    (void)hipEventDestroy(e);
    HISQ_HIP(r);
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

thread_local bool t_prof_suppressed = false;

bool profile_enabled() { return g_prof_on && !t_prof_suppressed; }

ProfileSuppress::ProfileSuppress() : prev_(t_prof_suppressed) { t_prof_suppressed = true; }
ProfileSuppress::~ProfileSuppress() { t_prof_suppressed = prev_; }

extern int64_t g_gemm_f32;  // gemm.hip

// "cg_multi_graph": -1 automatic (off), 0 off, 1: hisq_cg_solve_multi
// launches the chunks of all systems as one graph (ChunkGroup).
int64_t g_multi_graph = -1;
bool cg_multi_graph() { return g_multi_graph == 1 && !g_prof_on; }

// "cg_reliable_freeze": -1 automatic, 0 off, 1 on (see ru_freeze in CgDev).
int64_t g_ru_freeze = -1;

// "cg_graphs": -1 automatic, 0 off, 1 on (never while kernel timing is on:
// its events would be captured into the graph).
int64_t g_cg_graphs = -1;

bool cg_use_graphs(const hisq_gauge_s *g, int nrhs) {
    (void)g;
    (void)nrhs;
    // Measured on MI355X: replaying captured chunks does not shorten an
    // iteration (34 us at 8^4 with one RHS, 150 us at 16^3 x 32 with 12 RHS,
    // either way: the five dependent kernels, not the host, set the pace), so
    // automatic means off.
    return g_cg_graphs == 1 && !g_prof_on;
}

ProfileScope::ProfileScope(const char *cls, hipStream_t s) : s_(s), cls_(cls) {
    if (!g_prof_on || t_prof_suppressed) return;
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
    if (std::string(key) == "gemm_fp32_mfma") {
        if (value != -1 && value != 0 && value != 1)
            return fail(HISQ_ERR_INVALID_ARG, "gemm_fp32_mfma must be -1, 0 or 1");
        g_gemm_f32 = value;
        return HISQ_OK;
    }
    if (std::string(key) == "cg_multi_graph") {
        if (value != -1 && value != 0 && value != 1)
            return fail(HISQ_ERR_INVALID_ARG, "cg_multi_graph must be -1, 0 or 1");
        g_multi_graph = value;
        return HISQ_OK;
    }
    if (std::string(key) == "cg_reliable_freeze") {
        if (value != -1 && value != 0 && value != 1)
            return fail(HISQ_ERR_INVALID_ARG, "cg_reliable_freeze must be -1, 0 or 1");
        g_ru_freeze = value;
        return HISQ_OK;
    }
    if (std::string(key) == "cg_graphs") {
        if (value != -1 && value != 0 && value != 1)
            return fail(HISQ_ERR_INVALID_ARG, "cg_graphs must be -1, 0 or 1");
        g_cg_graphs = value;
        return HISQ_OK;
    }
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
