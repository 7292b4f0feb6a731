// hisq_autotune_dslash: choose the half-stencil launch shape by timing every
// shape the kernel provides on this volume, batch size and precision.
#include <cmath>
#include <vector>

#include "dslash_kernel.h"

namespace hisq {
hisq_status check_gauge(hisq_gauge g);
hisq_status check_nrhs(int nrhs);
void dslash_tuned_set(int vh, int nrhs, size_t real_bytes, const DslashShape &sh);
hisq_status dslash_set_tuning(const std::string &key, int64_t value);
}  // namespace hisq

using namespace hisq;

namespace {

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Restores the process-wide knobs on every exit path.
struct KnobGuard {
    ~KnobGuard() {
        (void)dslash_set_tuning("dslash_rhs_per_thread", 0);
        (void)dslash_set_tuning("dslash_lanes_per_site", 0);
        (void)dslash_set_tuning("dslash_group_order", -1);
        (void)dslash_set_tuning("dslash_xcd_remap", -1);
        (void)dslash_set_tuning("dslash_march", -1);
        (void)dslash_set_tuning("dslash_blocks_per_cu", -1);
    }
};

}  // namespace

extern "C" hisq_status hisq_autotune_dslash(hisq_gauge g, int nrhs, hisq_prec prec, int reps,
                                            hisq_tune_result *result_host, void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    if (prec != HISQ_FP64 && prec != HISQ_FP32)
        return fail(HISQ_ERR_INVALID_ARG, "prec must be HISQ_FP64 or HISQ_FP32");
    if (reps < 0) return fail(HISQ_ERR_INVALID_ARG, "reps must be >= 0");
    if (reps == 0) reps = 20;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int vh = g->geom.vh;
    const size_t rb = prec == HISQ_FP64 ? 8 : 4;
    const size_t bytes = 2 * rb * 3 * (size_t)vh * nrhs;
    void *pin = nullptr, *pout = nullptr;
    HISQ_TRY(g->ws.get("tune_in", bytes, &pin));
    HISQ_TRY(g->ws.get("tune_out", bytes, &pout));
    HISQ_HIP(hipMemsetAsync(pin, 0, bytes, s));
    EventPair ev;
    HISQ_HIP(hipEventCreate(&ev.a));
    HISQ_HIP(hipEventCreate(&ev.b));
    KnobGuard guard;

    auto launch = [&]() -> hisq_status {
        if (prec == HISQ_FP64)
            return launch_dslash(g, 0, static_cast<const double2 *>(pin),
                                 static_cast<double2 *>(pout), nrhs, nullptr, 0.0, nullptr, 0.0, 1.0,
                                 FIN_NONE, nullptr, nullptr, s);
        return launch_dslash_f32(g, 0, static_cast<const float2 *>(pin), static_cast<float2 *>(pout),
                                 nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, nullptr, s);
    };
    auto time_current = [&](double *us) -> hisq_status {
        for (int w = 0; w < 2; ++w) HISQ_TRY(launch());
        HISQ_HIP(hipEventRecord(ev.a, s));
        for (int r = 0; r < reps; ++r) HISQ_TRY(launch());
        HISQ_HIP(hipEventRecord(ev.b, s));
        HISQ_HIP(hipEventSynchronize(ev.b));
        float ms = 0.f;
        HISQ_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        *us = 1e3 * ms / reps;
        return HISQ_OK;
    };

    // the shape in use before tuning (built-in default or an earlier choice)
    DslashShape def = dslash_pick_shape(nrhs, vh, rb, false, g->geom);
    double us_def = 0.0;
    HISQ_TRY(dslash_set_tuning("dslash_rhs_per_thread", def.nr));
    HISQ_TRY(dslash_set_tuning("dslash_lanes_per_site", def.lps));
    HISQ_TRY(dslash_set_tuning("dslash_group_order", def.group_outer));
    HISQ_TRY(dslash_set_tuning("dslash_xcd_remap", def.xcd_remap));
    HISQ_TRY(dslash_set_tuning("dslash_march", def.march));
    HISQ_TRY(dslash_set_tuning("dslash_blocks_per_cu", def.blocks_per_cu));
    HISQ_TRY(time_current(&us_def));
    HISQ_TRY(dslash_set_tuning("dslash_blocks_per_cu", 0));
    const int kind = rb == 8 ? 0 : 1;
    const bool march_geom = (int64_t)g->geom.Xh * g->geom.Y * g->geom.Z % 256 == 0;

    const int nr1[] = {1, 2, 3, 4, 6, 12}, nrn[] = {1, 3, 6};
    DslashShape best = def;
    double us_best = us_def;
    int timed = 1;
    for (int lps : {1, 2, 4}) {
        const int *opts = lps == 1 ? nr1 : nrn;
        const int nopt = lps == 1 ? 6 : 3;
        for (int i = 0; i < nopt; ++i) {
            const int nr = opts[i];
            // groups much wider than the batch only add idle lanes
            if (nr * lps > 2 * nrhs && !(nr == 1 && lps == 1)) continue;
            if (!dslash_impl::shape_fits(nr, lps, vh, 6 * rb)) continue;
            const int ngroups = (nrhs + nr * lps - 1) / (nr * lps);
            for (int order = 0; order < (ngroups > 1 ? 2 : 1); ++order) {
                // dispatch order, contiguous ranges, or chunks of an eighth
                // of a time slice per XCD
                const int chunk = xcd_chunk_blocks(g->geom, ngroups);
                for (int xi = 0; xi < 3; ++xi) {
                    const int xcd = xi < 2 ? xi : chunk;
                    HISQ_TRY(dslash_set_tuning("dslash_rhs_per_thread", nr));
                    HISQ_TRY(dslash_set_tuning("dslash_lanes_per_site", lps));
                    HISQ_TRY(dslash_set_tuning("dslash_group_order", order));
                    HISQ_TRY(dslash_set_tuning("dslash_xcd_remap", xcd));
                    HISQ_TRY(dslash_set_tuning("dslash_march", 0));
                    double us = 0.0;
                    HISQ_TRY(time_current(&us));
                    ++timed;
                    if (us < us_best) {
                        us_best = us;
                        best = DslashShape{nr, lps, xcd, order};
                    }
                }
            }
            // the time-marching kernel with this shape (time segments chosen
            // automatically, XCD-contiguous chunks)
            if (march_geom && nrhs >= 2 && dslash_impl::march_shape_supported(kind, nr, lps)) {
                HISQ_TRY(dslash_set_tuning("dslash_rhs_per_thread", nr));
                HISQ_TRY(dslash_set_tuning("dslash_lanes_per_site", lps));
                HISQ_TRY(dslash_set_tuning("dslash_group_order", 0));
                HISQ_TRY(dslash_set_tuning("dslash_xcd_remap", 1));
                HISQ_TRY(dslash_set_tuning("dslash_march", 0));
                const DslashShape auto_m = [&] {
                    (void)dslash_set_tuning("dslash_march", -1);
                    return dslash_pick_shape(nrhs, vh, rb, false, g->geom);
                }();
                const int nseg = auto_m.march > 0 ? auto_m.march : 4;
                HISQ_TRY(dslash_set_tuning("dslash_march", nseg));
                double us = 0.0;
                HISQ_TRY(time_current(&us));
                ++timed;
                if (us < us_best) {
                    us_best = us;
                    best = DslashShape{nr, lps, 1, 0};
                    best.march = nseg;
                }
            }
        }
    }
    // then a cap on the blocks per compute unit for the best shape (fewer
    // sites in flight per XCD can keep more of the neighbour gathers in L2)
    if (best.march == 0) {
        HISQ_TRY(dslash_set_tuning("dslash_rhs_per_thread", best.nr));
        HISQ_TRY(dslash_set_tuning("dslash_lanes_per_site", best.lps));
        HISQ_TRY(dslash_set_tuning("dslash_group_order", best.group_outer));
        HISQ_TRY(dslash_set_tuning("dslash_xcd_remap", best.xcd_remap));
        HISQ_TRY(dslash_set_tuning("dslash_march", 0));
        for (int cap : {4, 3, 2}) {
            HISQ_TRY(dslash_set_tuning("dslash_blocks_per_cu", cap));
            double us = 0.0;
            HISQ_TRY(time_current(&us));
            ++timed;
            if (us < us_best) {
                us_best = us;
                best.blocks_per_cu = cap;
            }
        }
        HISQ_TRY(dslash_set_tuning("dslash_blocks_per_cu", -1));
    }
    dslash_tuned_set(vh, nrhs, rb, best);
    if (result_host) {
        *result_host = hisq_tune_result{};
        result_host->rhs_per_thread = best.nr;
        result_host->lanes_per_site = best.lps;
        result_host->group_order = best.group_outer;
        result_host->xcd_remap = best.xcd_remap;
        result_host->us_best = us_best;
        result_host->us_default = us_def;
        result_host->shapes_timed = timed;
        result_host->blocks_per_cu = best.blocks_per_cu;
        result_host->march = best.march;
    }
    return HISQ_OK;
}
