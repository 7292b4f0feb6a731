// FP64 half stencil launches, the launch-shape knobs and M^H M.  The kernel
// itself is in dslash_kernel.h.
#include "dslash_kernel.h"

namespace hisq {

// Process-wide launch-shape knobs (hisq_set_tuning).
struct DslashTuning {
    int64_t rhs_per_thread = 0;
    int64_t group_order = 0;
    int64_t xcd_remap = 1;
};
DslashTuning g_tune;
int64_t dslash_tune_xcd_remap() { return g_tune.xcd_remap; }
int64_t dslash_tune_group_order() { return g_tune.group_order; }

// Right-hand sides per thread: the tuned value, else measured defaults.  With
// many RHS the input field no longer fits the per-XCD L2 and the neighbour
// gathers are served from the last-level cache; then occupancy (latency
// hiding) matters more than link reuse in registers: 2 per thread up to
// Vh = 2^18 (16^3 x 32 with 12 RHS: 78 us against 93 us with 4), 3 above
// (32^3 x 64: 1.68 ms against 1.74 ms).  A group may be partly empty; lanes
// mask r < nr.
int dslash_pick_nr(int nrhs, int vh) {
    if (g_tune.rhs_per_thread > 0) return (int)g_tune.rhs_per_thread;
    if (nrhs <= 2) return nrhs;
    if (nrhs <= 4) return nrhs;
    return vh <= (1 << 18) ? 2 : 3;
}


hisq_status dslash_set_tuning(const std::string &key, int64_t v) {
    if (key == "dslash_rhs_per_thread") {
        if (!(v == 0 || v == 1 || v == 2 || v == 3 || v == 4 || v == 6 || v == 12))
            return fail(HISQ_ERR_INVALID_ARG, "dslash_rhs_per_thread must be 0, 1, 2, 3, 4, 6 or 12");
        g_tune.rhs_per_thread = v;
    } else if (key == "dslash_group_order") {
        if (v != 0 && v != 1) return fail(HISQ_ERR_INVALID_ARG, "dslash_group_order must be 0 or 1");
        g_tune.group_order = v;
    } else if (key == "dslash_xcd_remap") {
        if (v != 0 && v != 1) return fail(HISQ_ERR_INVALID_ARG, "dslash_xcd_remap must be 0 or 1");
        g_tune.xcd_remap = v;
    } else {
        return fail(HISQ_ERR_INVALID_ARG, "unknown tuning key '" + key + "'");
    }
    return HISQ_OK;
}

int dslash_reduce_blocks(const hisq_gauge_s *g, int nrhs) {
    (void)nrhs;
    return (g->geom.vh + dslash_impl::kBS - 1) / dslash_impl::kBS;
}

hisq_status launch_dslash(const hisq_gauge_s *g, int out_parity, const double2 *in,
                          double2 *out, int nrhs, const double2 *aux, double ca,
                          const double2 *aux2, double cb, double cd, DslashFinal fin,
                          const CgDev *cg, const Reduce *red, hipStream_t s) {
    (void)cg;
    using V = vec2<double>;
    const V *fat[2] = {reinterpret_cast<const V *>(g->fat[0]), reinterpret_cast<const V *>(g->fat[1])};
    const V *lng[2] = {reinterpret_cast<const V *>(g->lng[0]), reinterpret_cast<const V *>(g->lng[1])};
    ProfileScope prof(aux2 ? "dslash_aux2" : aux ? "dslash_aux" : "dslash", s);
    return dslash_impl::launch_dslash_t<double>(
        g->geom, fat, lng, out_parity, reinterpret_cast<const V *>(in), reinterpret_cast<V *>(out),
        nrhs, reinterpret_cast<const V *>(aux), ca, reinterpret_cast<const V *>(aux2), cb, cd,
        fin == FIN_CG_ALPHA ? red->partials : nullptr, dslash_pick_nr(nrhs, g->geom.vh),
        (int)g_tune.xcd_remap, (int)g_tune.group_order, s);
}

hisq_status apply_mdagm(hisq_gauge_s *g, double two_m, const double2 *in, double2 *out,
                        int nrhs, hipStream_t s) {
    void *tmp = nullptr;
    HISQ_TRY(g->ws.get("mdagm_tmp", sizeof(double2) * 3 * (size_t)g->geom.vh * nrhs, &tmp));
    double2 *t = static_cast<double2 *>(tmp);
    HISQ_TRY(launch_dslash(g, 1, in, t, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE,
                           nullptr, nullptr, s));
    HISQ_TRY(launch_dslash(g, 0, t, out, nrhs, in, two_m * two_m, nullptr, 0.0, -1.0, FIN_NONE,
                           nullptr, nullptr, s));
    return HISQ_OK;
}

}  // namespace hisq
