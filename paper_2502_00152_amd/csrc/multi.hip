// hisq_cg_solve_multi: independent CG solves on several lattices and masses
// at once.  Small lattices leave most of the GPU idle between the five
// dependent kernels of an iteration; solving several systems concurrently
// (one host thread and one stream per gauge handle) fills those gaps.
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "hisq_internal.h"

namespace hisq {
hisq_status check_gauge(hisq_gauge g);
}  // namespace hisq

using namespace hisq;

extern "C" hisq_status hisq_cg_solve_multi(int n_systems, const hisq_system *systems,
                                           const hisq_cg_params *params,
                                           hisq_cg_stats *stats_host, void *stream) {
    if (n_systems < 1) return fail(HISQ_ERR_INVALID_ARG, "n_systems must be >= 1");
    if (!systems || !params) return fail(HISQ_ERR_INVALID_ARG, "systems and params must be set");
    std::vector<int64_t> offset(n_systems + 1, 0);
    std::map<hisq_gauge, std::vector<int>> by_handle;
    std::vector<hisq_gauge> order;  // handles in order of first appearance
    for (int i = 0; i < n_systems; ++i) {
        HISQ_TRY(check_gauge(systems[i].g));
        if (systems[i].reserved) return fail(HISQ_ERR_INVALID_ARG, "reserved fields must be 0");
        if (systems[i].nrhs < 1) return fail(HISQ_ERR_INVALID_ARG, "nrhs must be >= 1");
        offset[i + 1] = offset[i] + systems[i].nrhs;
        auto &v = by_handle[systems[i].g];
        if (v.empty()) order.push_back(systems[i].g);
        v.push_back(i);
    }
    struct Outcome {
        hisq_status st = HISQ_OK;
        std::string msg;
    };
    std::vector<Outcome> out(n_systems);
    // one graph per chunk for all systems, if asked for (one device, no
    // kernel timing: its events would be captured)
    bool one_device = true;
    for (hisq_gauge g : order) one_device = one_device && g->device == order[0]->device;
    const bool combined = order.size() > 1 && one_device && cg_multi_graph();
    ChunkGroup group((int)order.size());
    auto run_group = [&](hisq_gauge g) {
        struct Member {  // leaves the group when the thread has no system left
            ChunkGroup *grp;
            ~Member() {
                if (grp) grp->leave();
                t_chunk_group = nullptr;
                t_chunk_sys = -1;
            }
        } member{combined ? &group : nullptr};
        t_chunk_group = member.grp;
        if (hipSetDevice(g->device) != hipSuccess) {
            for (int i : by_handle[g]) out[i] = {HISQ_ERR_HIP, "hipSetDevice failed"};
            return;
        }
        for (int i : by_handle[g]) {
            t_chunk_sys = i;
            const hisq_system &S = systems[i];
            const hisq_status st =
                hisq_cg_solve(S.g, S.two_m, S.b_dev, S.x_dev, S.nrhs, &params[i],
                              stats_host ? stats_host + offset[i] : nullptr, stream);
            out[i].st = st;
            if (st != HISQ_OK) out[i].msg = hisq_last_error();
        }
    };
    if (order.size() == 1) {
        run_group(order[0]);
    } else {
        std::vector<std::thread> threads;
        threads.reserve(order.size());
        for (hisq_gauge g : order) threads.emplace_back(run_group, g);
        for (auto &t : threads) t.join();
    }
    for (int i = 0; i < n_systems; ++i)
        if (out[i].st != HISQ_OK)
            return fail(out[i].st, "system " + std::to_string(i) + ": " + out[i].msg);
    return HISQ_OK;
}
