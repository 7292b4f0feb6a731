// FP64 half stencil launches, the launch-shape knobs and M^H M.  The kernel
// itself is in dslash_kernel.h.
#include "dslash_kernel.h"

namespace hisq {

// Process-wide launch-shape knobs (hisq_set_tuning).
struct DslashTuning {
    int64_t rhs_per_thread = 0;
    int64_t lanes_per_site = 0;
    int64_t group_order = -1;
    int64_t xcd_remap = -1;
    int64_t march = -1;  // time-marching kernel: -1 automatic, 0 off, n > 0 n time segments
    int64_t blocks_per_cu = -1;  // -1 automatic, 0 no cap, n > 0 at most n blocks per CU
};
DslashTuning g_tune;

// Shapes chosen by the autotuner, keyed by (Vh, nrhs, bytes per real).
struct TunedKey {
    int vh, nrhs, rb;
    bool operator<(const TunedKey &o) const {
        return vh != o.vh ? vh < o.vh : nrhs != o.nrhs ? nrhs < o.nrhs : rb < o.rb;
    }
};
std::map<TunedKey, DslashShape> g_tuned;

void dslash_tuned_set(int vh, int nrhs, size_t real_bytes, const DslashShape &sh) {
    g_tuned[TunedKey{vh, nrhs, (int)real_bytes}] = sh;
}
void dslash_tuned_clear() { g_tuned.clear(); }

namespace {
bool supported_shape(int nr, int lps) {
    if (lps == 1) return nr == 1 || nr == 2 || nr == 3 || nr == 4 || nr == 6 || nr == 12;
    if (lps == 2 || lps == 4) return nr == 1 || nr == 3 || nr == 6;
    return false;
}

// Smallest supported NR for lps lanes per site that covers nrhs in one group,
// else the largest.
int nr_for(int nrhs, int lps) {
    const int opts1[] = {1, 2, 3, 4, 6, 12}, optsn[] = {1, 3, 6};
    const int *o = lps == 1 ? opts1 : optsn;
    const int n = lps == 1 ? 6 : 3;
    for (int i = 0; i < n; ++i)
        if (o[i] * lps >= nrhs) return o[i];
    return o[n - 1];
}
}  // namespace

// Launch shape of the half stencil for nrhs RHS at half volume vh in the
// given precision: the tuned values where set, else defaults measured on
// MI355X (16^3 x 32 to 48^3 x 96, 1 to 24 RHS).  One RHS streams at 73-76% of
// HBM peak either way; with several RHS per site the links are read once per
// group and the sites of a block spread over the XCD's L2.  Measured with 12
// and 24 RHS: FP32 vectors with 16-bit links run best (or within 10%) with 3
// RHS per lane at every volume; FP32 links with 3 per lane on small volumes
// and up to 12 per lane on large ones (the (6 per lane, 4 lanes) shape chosen
// earlier for 32^3 x 64 was up to 1.6x slower elsewhere); FP64 with 2 lanes
// of 3 RHS (M^H M with 12 RHS at 16^3 x 32: 139 us against 162-175 us with 4
// lanes of 1 RHS; 24 RHS at 32^3 x 64: 5.3 ms against 5.8 ms with 12 RHS per
// lane), the lanes loading the next hop before the current hop's arithmetic.
// q16_links selects the 16-bit-link defaults (FP32 vectors, real_bytes 4).
// Geometries the time-marching kernel handles: whole 256-site chunks per time slice.
bool geom_march_ok(const Geom &g) {
    return g.T >= 2 && (int64_t)g.Xh * g.Y * g.Z % dslash_impl::kSites == 0;
}

// XCD remap value meaning "chunks of one eighth of a time slice" (resolved
// once the RHS groups are known).
constexpr int kXcdChunkAuto = -2;

// Chunks of site blocks dealt round-robin to the XCDs, one eighth of a time
// slice each (times the RHS groups of a site block), so that the eight XCDs
// sweep one time slice per round together: the time and z neighbours of the
// sites in flight are then shared in the last-level cache.  Measured with 12
// RHS (HIP events, including the 16-bit format conversions): 16-bit vectors
// 0.600 -> 0.537 ms at 32^3 x 64 and 3.11 -> 2.74 ms at 48^3 x 96, FP32 0.743
// -> 0.661 and 3.83 -> 3.59 ms, FP64 1.475 -> 1.233 and 7.16 -> 6.50 ms
// against one contiguous range per XCD; one RHS is unchanged or slower, so
// it keeps the contiguous ranges.
int xcd_chunk_blocks(const Geom &geom, int ngroups) {
    const int64_t S = (int64_t)geom.Xh * geom.Y * geom.Z;
    const int64_t c = (S + 8 * dslash_impl::kSites - 1) / (8 * dslash_impl::kSites);
    return (int)std::max<int64_t>(2, std::min<int64_t>(c * ngroups, 1 << 20));
}

DslashShape dslash_pick_shape(int nrhs, int vh, size_t real_bytes, bool q16_links,
                              const Geom &geom, bool plain) {
    const bool f32 = real_bytes <= 4, small = vh <= (1 << 18);  // FP32 and BF16
    DslashShape sh{};
    int xcd = nrhs >= 3 && !small ? kXcdChunkAuto : 1;
    if (nrhs <= 2) {
        sh.nr = nrhs, sh.lps = 1, xcd = f32 ? 0 : 1;
    } else if (nrhs <= 4) {
        sh.nr = 2, sh.lps = 1;
    } else if (f32) {
        // large volumes: 6 RHS per lane for FP32 vectors and for 16-bit links
        // (M^H M with 24 RHS at 32^3 x 64: 16-bit vectors 2.13 against 2.39
        // ms with 3 per lane, FP32 with 16-bit links 2.46 against 2.63, FP32
        // 2.83 against 2.94 with 12 per lane); BF16 keeps up to 12 per lane
        if (small) sh.nr = 3, sh.lps = 1;
        // packed 16-bit vectors without an epilogue field, 7-12 RHS: one
        // group of up to 12 per lane, the links read once (the CG's D_oe p at
        // 48^3 x 96: 1644 against 1697 us; with the field's registers the
        // launch with the epilogue is faster at 6: 1873 against 1917 us)
        else if (q16_links && real_bytes == 2 && plain && nrhs > 6 && nrhs <= 12)
            sh.nr = 12, sh.lps = 1;
        else if (q16_links || real_bytes == 4) sh.nr = nrhs >= 6 ? 6 : 3, sh.lps = 1;
        else sh.nr = nr_for(nrhs, 1), sh.lps = 1;
    } else {
        sh.nr = 3, sh.lps = 2;
    }
    int order = 0;
    // FP32 vectors (FP32 or 16-bit links) with 12 or more RHS on large
    // volumes: at most 3 blocks per CU (12 and 24 RHS: 3-5% faster at 32^3 x
    // 64, 5-10% at 48^3 x 96; 6 RHS unchanged)
    int cap = real_bytes == 4 && !small && nrhs >= 12 ? 3 : 0;
    // the autotuner's choice for this volume and batch, if any
    const auto it = g_tuned.find(TunedKey{vh, nrhs, q16_links ? 3 : (int)real_bytes});
    const bool tuned = it != g_tuned.end();
    if (tuned) {
        sh.nr = it->second.nr, sh.lps = it->second.lps;
        xcd = it->second.xcd_remap, order = it->second.group_outer;
        cap = it->second.blocks_per_cu;
    }
    // explicit knobs override both
    if (g_tune.rhs_per_thread > 0 || g_tune.lanes_per_site > 0) {
        cap = 0;  // a tuned cap belongs to the tuned shape
        sh.lps = g_tune.lanes_per_site > 0 ? (int)g_tune.lanes_per_site : 1;
        sh.nr = g_tune.rhs_per_thread > 0 ? (int)g_tune.rhs_per_thread : nr_for(nrhs, sh.lps);
    }
    sh.xcd_remap = g_tune.xcd_remap >= 0 ? (int)g_tune.xcd_remap : xcd;
    sh.group_outer = g_tune.group_order >= 0 ? (int)g_tune.group_order : order;
    sh.march = 0;
    const int kind = real_bytes == 8 ? 0 : real_bytes == 4 ? 1 : q16_links ? 2 : -1;
    if (tuned && g_tune.march < 0 && !(g_tune.rhs_per_thread > 0 || g_tune.lanes_per_site > 0)) {
        sh.march = it->second.march;
    } else if (kind >= 0 && nrhs >= 2 && g_tune.march != 0 && geom_march_ok(geom)) {
        // the time-marching kernel, when asked for: measured at 32^3 x 64 and
        // 48^3 x 96 with 12 RHS it cuts the bytes fetched beyond L2 by 10-30%
        // but runs no faster than this kernel (16-bit vectors 2.42 against
        // 2.31 ms, FP32 vectors with 16-bit links 3.19 against 3.18 ms at
        // 48^3 x 96), so it is off by default
        const bool want = g_tune.march > 0;
        if (want) {
            DslashShape m = sh;
            if (g_tune.rhs_per_thread > 0 || g_tune.lanes_per_site > 0) {
                m.nr = sh.nr, m.lps = sh.lps;  // explicit knobs
            } else if (kind == 0) {
                m.nr = 1, m.lps = 2;  // FP64: the ring of 3 RHS per lane spills
            } else {
                m.nr = 3, m.lps = 2;  // 6 RHS per group: no register spills
            }
            if (dslash_impl::march_shape_supported(kind, m.nr, m.lps)) {
                const int rg = m.nr * m.lps, ngroups = (nrhs + rg - 1) / rg;
                const int nchunk = geom.Xh * geom.Y * geom.Z / dslash_impl::kSites;
                const int nsteps = geom.T / 2;
                int nseg = (int)g_tune.march;
                if (nseg <= 0) {
                    // about 1024 workgroups, at least 4 steps per segment
                    nseg = (1024 + 2 * nchunk * ngroups - 1) / (2 * nchunk * ngroups);
                    nseg = std::max(1, std::min(nseg, nsteps / 4));
                }
                m.march = nseg;
                m.xcd_remap = 1;
                sh = m;
            }
        }
    }
    // the per-lane 32-bit offsets must cover the group: shrink it if not
    // (one RHS's colour vector at one site: 6 reals, or 16 bytes packed 16-bit)
    const size_t site_bytes = q16_links && real_bytes == 2 ? 16 : 6 * real_bytes;
    while (!dslash_impl::shape_fits(sh.nr, sh.lps, vh, site_bytes) && (sh.lps > 1 || sh.nr > 1)) {
        if (sh.lps > 1) sh.lps /= 2;
        else sh.nr = sh.nr == 12 ? 6 : sh.nr == 6 ? 3 : 1;
    }
    if (sh.xcd_remap == kXcdChunkAuto)
        sh.xcd_remap = xcd_chunk_blocks(geom, (nrhs + sh.nr * sh.lps - 1) / (sh.nr * sh.lps));
    sh.blocks_per_cu = g_tune.blocks_per_cu >= 0 ? (int)g_tune.blocks_per_cu : cap;
    return sh;
}

hisq_status dslash_check_shape(const DslashShape &sh) {
    // the time-marching kernel checks its own shapes per storage type
    if (sh.march > 0) return HISQ_OK;
    if (!supported_shape(sh.nr, sh.lps))
        return fail(HISQ_ERR_INVALID_ARG,
                    "dslash: unsupported (rhs_per_thread, lanes_per_site) = (" +
                        std::to_string(sh.nr) + ", " + std::to_string(sh.lps) + ")");
    return HISQ_OK;
}

hisq_status dslash_set_tuning(const std::string &key, int64_t v) {
    if (key == "dslash_rhs_per_thread") {
        if (!(v == 0 || v == 1 || v == 2 || v == 3 || v == 4 || v == 6 || v == 12))
            return fail(HISQ_ERR_INVALID_ARG, "dslash_rhs_per_thread must be 0, 1, 2, 3, 4, 6 or 12");
        g_tune.rhs_per_thread = v;
    } else if (key == "dslash_lanes_per_site") {
        if (!(v == 0 || v == 1 || v == 2 || v == 4))
            return fail(HISQ_ERR_INVALID_ARG, "dslash_lanes_per_site must be 0, 1, 2 or 4");
        g_tune.lanes_per_site = v;
    } else if (key == "dslash_group_order") {
        if (v != -1 && v != 0 && v != 1)
            return fail(HISQ_ERR_INVALID_ARG, "dslash_group_order must be -1, 0 or 1");
        g_tune.group_order = v;
    } else if (key == "dslash_autotune_clear") {
        dslash_tuned_clear();
    } else if (key == "dslash_march") {
        if (v < -1) return fail(HISQ_ERR_INVALID_ARG, "dslash_march must be -1, 0 or a segment count");
        g_tune.march = v;
    } else if (key == "dslash_blocks_per_cu") {
        if (v < -1 || v > dslash_impl::kMaxBlocksPerCu)
            return fail(HISQ_ERR_INVALID_ARG, "dslash_blocks_per_cu must be in [-1, 8]");
        g_tune.blocks_per_cu = v;
    } else if (key == "dslash_xcd_remap") {
        if (v < -1 || v > (1 << 20))
            return fail(HISQ_ERR_INVALID_ARG, "dslash_xcd_remap must be -1, 0, 1 or a chunk size");
        g_tune.xcd_remap = v;
    } else {
        return fail(HISQ_ERR_INVALID_ARG, "unknown tuning key '" + key + "'");
    }
    return HISQ_OK;
}

int dslash_reduce_blocks(const hisq_gauge_s *g, int nrhs) {
    (void)nrhs;
    return (g->geom.vh + dslash_impl::kSites - 1) / dslash_impl::kSites;
}

hisq_status launch_dslash(const hisq_gauge_s *g, int out_parity, const double2 *in,
                          double2 *out, int nrhs, const double2 *aux, double ca,
                          const double2 *aux2, double cb, double cd, DslashFinal fin,
                          const CgDev *cg, const Reduce *red, hipStream_t s,
                          const double *ca_rhs) {
    using V = vec2<double>;
    const V *fat[2] = {reinterpret_cast<const V *>(g->fat[0]), reinterpret_cast<const V *>(g->fat[1])};
    const V *lng[2] = {reinterpret_cast<const V *>(g->lng[0]), reinterpret_cast<const V *>(g->lng[1])};
    const DslashShape sh = dslash_pick_shape(nrhs, g->geom.vh, sizeof(double), false, g->geom);
    HISQ_TRY(dslash_check_shape(sh));
    ProfileScope prof(aux2 ? "dslash_aux2" : aux ? "dslash_aux" : "dslash", s);
    return dslash_impl::launch_dslash_t<double>(
        g->geom, fat, lng, out_parity, reinterpret_cast<const V *>(in), reinterpret_cast<V *>(out),
        nrhs, reinterpret_cast<const V *>(aux), ca, reinterpret_cast<const V *>(aux2), cb, cd,
        fin == FIN_CG_ALPHA ? red->partials : nullptr, sh, s, ca_rhs, cg ? cg->status : nullptr);
}

hisq_status apply_mdagm(hisq_gauge_s *g, double two_m, const double2 *in, double2 *out,
                        int nrhs, hipStream_t s, int parity, const double *m2_rhs,
                        const int *skip) {
    void *tmp = nullptr;
    HISQ_TRY(g->ws.get("mdagm_tmp", sizeof(double2) * 3 * (size_t)g->geom.vh * nrhs, &tmp));
    double2 *t = static_cast<double2 *>(tmp);
    // the stencil skips groups whose status entries are all non-active; skip
    // uses the same convention (0 = compute)
    CgDev sel{};
    sel.status = const_cast<int *>(skip);
    const CgDev *cg = skip ? &sel : nullptr;
    HISQ_TRY(launch_dslash(g, 1 - parity, in, t, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE,
                           cg, nullptr, s));
    HISQ_TRY(launch_dslash(g, parity, t, out, nrhs, in, two_m * two_m, nullptr, 0.0, -1.0,
                           FIN_NONE, cg, nullptr, s, m2_rhs));
    return HISQ_OK;
}

}  // namespace hisq
