// Mixed-precision CG with reliable updates and multi-deflation
// (arXiv:2502.00152: section 2, the conventional solve is mixed-precision CG;
// section 3, reliable updates with delta_rd and re-deflation with
// single-precision eigenvectors whenever the residual has fallen by 1/delta_tr
// since the last deflation).
//
// The recurrence runs on FP32 vectors with the FP32 operator (links in FP32,
// in BF16 at sloppy_prec = HISQ_BF16, or 16-bit fixed point at HISQ_Q16; at
// HISQ_HALF also p, A p and the odd temporary in 16-bit fixed point with a
// norm per site); its dot products and all scalars are FP64.  The solution accumulates in FP64: the FP32
// correction x_s is added to x at every reliable update, where the residual is
// recomputed in FP64 with the FP64 operator, r = b - A x, and replaces the
// iterated one.  A right-hand side gets a reliable update
//   - when its iterated residual falls below delta times the last true one
//     (the device flags it; the recurrence goes on until the host's next poll),
//   - optionally, after reliable_interval iterations since its last one,
//   - when its iterated residual meets the target (the convergence decision is
//     always taken on the FP64 true residual).
// Re-deflation (when enabled) runs at a reliable update whose true residual
// has fallen by tol_restart since the last deflation: x += V Lambda^-1 V^H r,
// r recomputed, and the recurrence restarted from p = r.
#include <cmath>
#include <vector>

#include "hisq_internal.h"

namespace hisq {
namespace {

struct Pinned {
    void *ptr = nullptr;
    ~Pinned() {
        if (ptr) (void)hipHostFree(ptr);
    }
};

template <typename T>
T *carve(char *&p, size_t count) {
    T *r = reinterpret_cast<T *>(p);
    p += ((sizeof(T) * count + 63) / 64) * 64;
    return r;
}

}  // namespace

hisq_status solve_mixed(hisq_gauge_s *g, double two_m, const double2 *b, double2 *x, int nrhs,
                        const hisq_cg_params *P, hisq_cg_stats *stats, hipStream_t s,
                        const double *m2_rhs, hisq_prec links) {
    const bool bf16_links = links == HISQ_BF16, q16_links = links == HISQ_Q16;
    // HISQ_HALF: p, A p and the odd temporary in 16-bit fixed point (one norm
    // per RHS and site, in the same buffers: 16 of their 24 bytes per site),
    // 16-bit links; r and the correction x_s stay FP32
    const bool half = links == HISQ_HALF;
    const int64_t vh = g->geom.vh;
    const int64_t n = 3 * (int64_t)g->geom.vh;
    const int interval = P->check_interval > 0 ? P->check_interval : 16;
    const int par = P->parity;
    const int ru_interval = P->reliable_interval;  // 0: delta trigger only
    const double delta = P->reliable_delta > 0.0 ? P->reliable_delta : 0.1;
    if (!(delta < 1.0)) return fail(HISQ_ERR_INVALID_ARG, "reliable_delta must be < 1");
    if (ru_interval < 0) return fail(HISQ_ERR_INVALID_ARG, "reliable_interval must be >= 0");
    const bool redefl = P->n_ev > 0 && P->tol_restart > 0.0;
    if (P->n_ev < 0) return fail(HISQ_ERR_INVALID_ARG, "n_ev must be >= 0");
    if (P->tol_restart < 0.0 || P->tol_restart >= 1.0)
        return fail(HISQ_ERR_INVALID_ARG, "tol_restart must be in [0, 1)");
    if (P->tol_restart > 0.0 && P->n_ev == 0)
        return fail(HISQ_ERR_INVALID_ARG, "tol_restart > 0 needs n_ev > 0 eigenvectors");
    std::vector<double> w;
    if (redefl) {
        if (!P->evecs_dev || !P->evals_host)
            return fail(HISQ_ERR_INVALID_ARG, "re-deflation needs evecs_dev and evals_host");
        if (P->n_ev > n) return fail(HISQ_ERR_INVALID_ARG, "n_ev must be <= 3*Vh");
        if (P->evec_prec != HISQ_FP64 && P->evec_prec != HISQ_FP32)
            return fail(HISQ_ERR_INVALID_ARG, "evec_prec must be HISQ_FP64 or HISQ_FP32");
        w.resize(P->n_ev);
        for (int i = 0; i < P->n_ev; ++i) {
            const double lam = P->evals_host[i] + two_m * two_m;
            if (!std::isfinite(lam) || !(lam > 0.0))
                return fail(HISQ_ERR_INVALID_ARG, "eps_i + (2m)^2 must be finite and > 0");
            w[i] = 1.0 / lam;
        }
    }

    // the sloppy links are made here, not inside a captured iteration chunk
    if (bf16_links) HISQ_TRY(ensure_links_bf16(g, s));
    else if (half) HISQ_TRY(ensure_links_q16n(g, s));
    else if (q16_links) HISQ_TRY(ensure_links_q16(g, s));
    else HISQ_TRY(ensure_links_f32(g, s));

    // ------------------------------------------------------------ buffers
    const size_t v64 = sizeof(double2) * (size_t)n * nrhs, v32 = sizeof(float2) * (size_t)n * nrhs;
    void *p = nullptr;
    HISQ_TRY(g->ws.get("cg_r", v64, &p));
    double2 *r = static_cast<double2 *>(p);
    HISQ_TRY(g->ws.get("cg_Ap", v64, &p));
    double2 *Ax = static_cast<double2 *>(p);
    HISQ_TRY(g->ws.get("cg_p", v64, &p));
    double2 *p64 = static_cast<double2 *>(p);  // written by cg_init only
    HISQ_TRY(g->ws.get("mx_rs", v32, &p));
    float2 *rs = static_cast<float2 *>(p);
    HISQ_TRY(g->ws.get("mx_ps", v32, &p));
    float2 *ps = static_cast<float2 *>(p);
    HISQ_TRY(g->ws.get("mx_Aps", v32, &p));
    float2 *Aps = static_cast<float2 *>(p);
    HISQ_TRY(g->ws.get("mx_xs", v32, &p));
    float2 *xs = static_cast<float2 *>(p);
    HISQ_TRY(g->ws.get("mx_t", v32, &p));
    float2 *t32 = static_cast<float2 *>(p);
    // device scalars: CgDev arrays + masks
    const size_t nd = 12, ni = 8;
    HISQ_TRY(g->ws.get("mx_scalars", (nd * sizeof(double) + ni * sizeof(int)) * nrhs + 64 * (nd + ni), &p));
    char *cp = static_cast<char *>(p);
    CgDev dev{};
    // The host mirror below is carved in the same order, so that the state a
    // poll reads (rho, status, iters, ru_flag) is one contiguous copy, and so
    // is what a reliable update writes back (those, rho_ru, true_res2, the
    // restart coefficients and modes).
    dev.rho = carve<double>(cp, nrhs);
    dev.status = carve<int>(cp, nrhs);
    dev.iters = carve<int>(cp, nrhs);
    dev.ru_flag = carve<int>(cp, nrhs);
    dev.rho_ru = carve<double>(cp, nrhs);
    dev.true_res2 = carve<double>(cp, nrhs);
    double *d_rbeta = carve<double>(cp, nrhs);
    int *d_mode = carve<int>(cp, nrhs);
    dev.rho_pend = carve<double>(cp, nrhs);
    dev.alpha = carve<double>(cp, nrhs);
    dev.beta = carve<double>(cp, nrhs);
    dev.bnorm2 = carve<double>(cp, nrhs);
    dev.tol2b = carve<double>(cp, nrhs);
    dev.xp_alpha = carve<double>(cp, nrhs);
    dev.xp_beta = carve<double>(cp, nrhs);
    double *d_rho_t = carve<double>(cp, nrhs);
    dev.checks = carve<int>(cp, nrhs);
    dev.xp_mode = carve<int>(cp, nrhs);
    int *d_mask = carve<int>(cp, nrhs);
    int *d_skip = carve<int>(cp, nrhs);
    dev.delta2 = delta * delta;
    // With BF16 links the sloppy operator is accurate to ~1e-3 only: a
    // recurrence run on past the delta trigger (until the next poll) can make
    // the FP64 correction diverge on ill-conditioned systems, so the RHS stops
    // at the trigger, as in the paper's reliable update.  FP32 and 16-bit
    // vectors go on: stopping lets the RHS of a batch trigger in separate
    // rounds of FP64 updates (measured on the 48^3 x 96 deflated solve, 12
    // RHS: 3.29 solves/s running on against 2.92 stopped, 566 and 571
    // iterations), though an undeflated ill-conditioned solve gains from it
    // (32^3 x 64, 2m = 0.005, 16-bit vectors: 1204 iterations stopped against
    // 1475, 1.69 against 2.18 s); "cg_reliable_freeze" chooses.
    dev.ru_freeze = g_ru_freeze >= 0 ? (int)g_ru_freeze : (bf16_links ? 1 : 0);
    dev.max_iter = P->max_iter;

    const int nb_pap = dslash_reduce_blocks(g, nrhs);
    const int nb_blas = blas_reduce_blocks(n);
    Reduce red{}, pap{};
    HISQ_TRY(g->ws.get("reduce_partials",
                       sizeof(double) * (size_t)nrhs *
                           std::max<int>(std::max(2 * nb_blas, nb_pap), mixed_resid_blocks(n)),
                       &p));
    red.partials = static_cast<double *>(p);
    HISQ_TRY(g->ws.get("cg_pap_partials", sizeof(double) * (size_t)nrhs * nb_pap, &p));
    pap.partials = static_cast<double *>(p);

    double *d_w = nullptr;
    double2 *d_C = nullptr;
    if (redefl) {
        HISQ_TRY(g->ws.get("deflate_w", sizeof(double) * P->n_ev, &p));
        d_w = static_cast<double *>(p);
        HISQ_TRY(g->ws.get("deflate_c", sizeof(double2) * (size_t)P->n_ev * nrhs, &p));
        d_C = static_cast<double2 *>(p);
        HISQ_HIP(hipMemcpyAsync(d_w, w.data(), sizeof(double) * P->n_ev, hipMemcpyHostToDevice, s));
    }

    // host mirror (pinned): doubles rho, rho_ru, rho_t, bnorm2, true_res2, rbeta; ints
    // status, iters, defl, mask, mode, ru_flag
    Pinned pin;
    HISQ_HIP(hipHostMalloc(&pin.ptr, (6 * sizeof(double) + 7 * sizeof(int)) * nrhs + 64 * 13,
                           hipHostMallocDefault));
    char *hp = static_cast<char *>(pin.ptr);
    double *h_rho = carve<double>(hp, nrhs);
    int *h_status = carve<int>(hp, nrhs), *h_iters = carve<int>(hp, nrhs);
    int *h_flag = carve<int>(hp, nrhs);
    const size_t poll_bytes = (size_t)(hp - static_cast<char *>(pin.ptr));
    double *h_rho_ru = carve<double>(hp, nrhs), *h_tr2 = carve<double>(hp, nrhs);
    double *h_rbeta = carve<double>(hp, nrhs);
    int *h_mode = carve<int>(hp, nrhs);
    const size_t state_bytes = (size_t)(hp - static_cast<char *>(pin.ptr));
    double *h_rho_t = carve<double>(hp, nrhs), *h_b2 = carve<double>(hp, nrhs);
    int *h_defl = carve<int>(hp, nrhs), *h_mask = carve<int>(hp, nrhs);
    int *h_skip = carve<int>(hp, nrhs);
    std::vector<int> ru_count(nrhs, 0), defl_count(nrhs, 0), iters_at_ru(nrhs, 0);
    std::vector<double> rho_defl(nrhs, 0.0);

    auto sync = [&]() -> hisq_status {
        HISQ_HIP(hipStreamSynchronize(s));
        return HISQ_OK;
    };
    auto d2h = [&](void *dst, const void *src, size_t bytes) -> hisq_status {
        HISQ_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
        return HISQ_OK;
    };
    auto h2d = [&](void *dst, const void *src, size_t bytes) -> hisq_status {
        HISQ_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
        return HISQ_OK;
    };
    const size_t dn = sizeof(double) * nrhs, in_ = sizeof(int) * nrhs;

    // ------------------------------------------------------------- start
    // r = b - A x0 in FP64; rho = ||r||^2; statuses
    HISQ_TRY(apply_mdagm(g, two_m, x, Ax, nrhs, s, par, m2_rhs));
    HISQ_TRY(cg_init(n, nrhs, b, Ax, r, p64, P->tol, dev, red, s));
    HISQ_HIP(hipMemcpyAsync(dev.rho_ru, dev.rho, dn, hipMemcpyDeviceToDevice, s));
    HISQ_TRY(mixed_to_f32(r, rs, n, nrhs, nullptr, s));
    if (half) HISQ_TRY(half_p_restart(vh, nrhs, ps, rs, nullptr, nullptr, s));
    else HISQ_HIP(hipMemcpyAsync(ps, rs, v32, hipMemcpyDeviceToDevice, s));
    HISQ_HIP(hipMemsetAsync(xs, 0, v32, s));
    HISQ_TRY(d2h(h_rho, dev.rho, dn));
    HISQ_TRY(d2h(h_b2, dev.bnorm2, dn));
    HISQ_TRY(d2h(h_status, dev.status, in_));
    HISQ_TRY(d2h(h_iters, dev.iters, in_));
    HISQ_HIP(hipMemsetAsync(dev.ru_flag, 0, in_, s));
    HISQ_TRY(sync());
    // the host owns rho_ru and true_res2 from here on
    for (int q = 0; q < nrhs; ++q) {
        rho_defl[q] = h_rho[q];
        h_rho_ru[q] = h_rho[q];
        h_tr2[q] = h_rho[q];
        h_flag[q] = 0;
    }
    const double tol2 = P->tol * P->tol;
    const double m2 = two_m * two_m;

    // the <p, A p> partials as the r update and the state kernel read them
    double *pq_sum = nullptr;
    if (nb_pap >= kPapPresum) {
        HISQ_TRY(g->ws.get("cg_pq", sizeof(double) * nrhs, &p));
        pq_sum = static_cast<double *>(p);
    }
    struct PapView {
        const double *p;
        int nb;
    };
    auto pap_view = [&]() { return pq_sum ? PapView{pq_sum, 1} : PapView{pap.partials, nb_pap}; };

    auto iterate = [&]() -> hisq_status {
        if (half) {
            HISQ_TRY(launch_dslash_h16(g, 1 - par, ps, t32, nrhs, nullptr, 0.0, 1.0, nullptr, s,
                                       nullptr, dev.status));
            HISQ_TRY(launch_dslash_h16(g, par, t32, Aps, nrhs, ps, m2, -1.0, pap.partials, s,
                                       m2_rhs, dev.status));
            const PapView pv = pap_view();
            if (pq_sum) HISQ_TRY(cg_sum_pap(nrhs, pap.partials, nb_pap, pq_sum, s));
            HISQ_TRY(half_update_r(vh, nrhs, rs, Aps, pv.p, pv.nb, dev, red, s));
            HISQ_TRY(cg_finalize(n, nrhs, pv.p, pv.nb, dev, red, s));
            HISQ_TRY(half_update_xp(vh, nrhs, xs, rs, ps, dev, s));
            return HISQ_OK;
        }
        if (bf16_links) {
            HISQ_TRY(launch_dslash_f32_bl(g, 1 - par, ps, t32, nrhs, nullptr, 0.0, 1.0, nullptr, s,
                                          nullptr, dev.status));
            HISQ_TRY(launch_dslash_f32_bl(g, par, t32, Aps, nrhs, ps, m2, -1.0, pap.partials, s,
                                          m2_rhs, dev.status));
        } else if (q16_links) {
            HISQ_TRY(launch_dslash_f32_q16(g, 1 - par, ps, t32, nrhs, nullptr, 0.0, 1.0, nullptr,
                                           s, nullptr, dev.status));
            HISQ_TRY(launch_dslash_f32_q16(g, par, t32, Aps, nrhs, ps, m2, -1.0, pap.partials, s,
                                           m2_rhs, dev.status));
        } else {
            HISQ_TRY(launch_dslash_f32(g, 1 - par, ps, t32, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0,
                                       nullptr, s, nullptr, dev.status));
            HISQ_TRY(launch_dslash_f32(g, par, t32, Aps, nrhs, ps, m2, nullptr, 0.0, -1.0,
                                       pap.partials, s, m2_rhs, dev.status));
        }
        const PapView pv = pap_view();
        if (pq_sum) HISQ_TRY(cg_sum_pap(nrhs, pap.partials, nb_pap, pq_sum, s));
        HISQ_TRY(cg_update_r(n, nrhs, rs, Aps, pv.p, pv.nb, dev, red, s));
        HISQ_TRY(cg_finalize(n, nrhs, pv.p, pv.nb, dev, red, s));
        HISQ_TRY(cg_update_xp(n, nrhs, xs, rs, ps, dev, s));
        return HISQ_OK;
    };

    // r = b - A x for the masked RHS, rho_t on the host
    // r = b - A x for the RHS with host_mask[q] != 0 (all if null); A x is
    // computed for those RHS groups only
    auto true_residual = [&](const int *mask_dev, const int *host_mask) -> hisq_status {
        const int *skip = nullptr;
        if (host_mask) {
            for (int q = 0; q < nrhs; ++q) h_skip[q] = host_mask[q] ? 0 : 1;
            HISQ_TRY(h2d(d_skip, h_skip, in_));
            skip = d_skip;
        }
        HISQ_TRY(apply_mdagm(g, two_m, x, Ax, nrhs, s, par, m2_rhs, skip));
        HISQ_TRY(mixed_resid(b, Ax, r, n, nrhs, mask_dev, d_rho_t, red, s));
        HISQ_TRY(d2h(h_rho_t, d_rho_t, dn));
        return sync();
    };

    const int64_t cap = 4 * (int64_t)P->max_iter + 4 * (int64_t)interval + 16;
    int64_t enqueued = 0;
    const bool graphs = cg_use_graphs(g, nrhs);
    GraphChunk chunk;
    const std::function<hisq_status()> chunk_body = [&]() -> hisq_status {
        for (int k = 0; k < interval; ++k) HISQ_TRY(iterate());
        return HISQ_OK;
    };
    // Right after a reliable update no iteration has run since the host wrote
    // the state back, so the host mirror is current and the poll is skipped.
    bool mirror_current = false;
    for (;;) {
        if (!mirror_current) {
            // rho, status, iters, ru_flag in one copy
            HISQ_TRY(d2h(h_rho, dev.rho, poll_bytes));
            HISQ_TRY(sync());
        }
        mirror_current = false;
        int nactive = 0, nru = 0;
        for (int q = 0; q < nrhs; ++q) {
            const int st = h_status[q];
            const bool want = st == CG_PENDING ||
                              (st == CG_ACTIVE &&
                               (h_flag[q] || (ru_interval > 0 &&
                                              h_iters[q] - iters_at_ru[q] >= ru_interval)));
            h_mask[q] = want ? 1 : 0;
            nru += want;
            nactive += st == CG_ACTIVE;
        }
        if (nru == 0) {
            if (nactive == 0 || P->max_iter == 0 || enqueued >= cap) break;
            if (t_chunk_group && enqueued > 0) {
                // with the other systems' chunks in one graph (the first chunk
                // runs eagerly, so that lazily made copies exist before any capture)
                HISQ_TRY(t_chunk_group->run(s, t_chunk_sys, chunk_body));
            } else if (graphs) {
                HISQ_TRY(chunk.run(s, chunk_body));
            } else {
                HISQ_TRY(chunk_body());
            }
            enqueued += interval;
            continue;
        }
        // ------------------------------------------------ reliable update
        HISQ_TRY(h2d(d_mask, h_mask, in_));
        HISQ_TRY(mixed_accum_x(x, xs, n, nrhs, d_mask, s));
        HISQ_TRY(true_residual(d_mask, h_mask));
        int ndefl = 0;
        for (int q = 0; q < nrhs; ++q) {
            h_defl[q] = 0;
            h_mode[q] = 0;
            h_rbeta[q] = 0.0;
            if (!h_mask[q]) continue;
            const double rt = h_rho_t[q];
            const int st = h_status[q];
            h_flag[q] = 0;
            ++ru_count[q];
            iters_at_ru[q] = h_iters[q];
            h_tr2[q] = rt;
            if (!std::isfinite(rt)) {
                h_status[q] = CG_NAN;
            } else if (rt <= tol2 * h_b2[q]) {
                h_status[q] = CG_CONVERGED;
            } else if (h_iters[q] >= P->max_iter) {
                h_status[q] = CG_MAXITER;
            } else if (redefl && rt <= P->tol_restart * P->tol_restart * rho_defl[q]) {
                h_defl[q] = 1;
                ++ndefl;
            } else {
                // continue from the true residual.  A pending RHS has not built
                // its next direction yet: p = r + beta p with beta = rho_true /
                // rho_old; an active one keeps p.
                h_mode[q] = st == CG_PENDING ? 1 : 0;
                h_rbeta[q] = rt / h_rho[q];
                h_rho[q] = rt;
                h_rho_ru[q] = rt;
                h_status[q] = CG_ACTIVE;
            }
        }
        HISQ_TRY(mixed_to_f32(r, rs, n, nrhs, d_mask, s));
        if (ndefl > 0) {
            // x += V diag(w) V^H r for the RHS in h_defl; the coefficients of
            // the others are zeroed, so their x is unchanged
            HISQ_TRY(h2d(d_mask, h_defl, in_));
            if (P->evec_prec == HISQ_FP32) {
                const float2 *V = static_cast<const float2 *>(P->evecs_dev);
                HISQ_TRY(gemm_tn(g, V, P->n_ev, r, nrhs, n, d_w, 1.0, d_C, s));
                HISQ_TRY(mixed_mask_rows(d_C, P->n_ev, nrhs, d_mask, s));
                HISQ_TRY(gemm_nn(V, P->n_ev, d_C, nrhs, n, 1.0, x, s));
            } else {
                const double2 *V = static_cast<const double2 *>(P->evecs_dev);
                HISQ_TRY(gemm_tn(g, V, P->n_ev, r, nrhs, n, d_w, 1.0, d_C, s));
                HISQ_TRY(mixed_mask_rows(d_C, P->n_ev, nrhs, d_mask, s));
                HISQ_TRY(gemm_nn(V, P->n_ev, d_C, nrhs, n, 1.0, x, s));
            }
            HISQ_TRY(true_residual(d_mask, h_defl));
            HISQ_TRY(mixed_to_f32(r, rs, n, nrhs, d_mask, s));
            for (int q = 0; q < nrhs; ++q) {
                if (!h_defl[q]) continue;
                const double rt = h_rho_t[q];
                ++defl_count[q];
                ++ru_count[q];
                rho_defl[q] = rt;
                h_tr2[q] = rt;
                if (!std::isfinite(rt)) {
                    h_status[q] = CG_NAN;
                } else if (rt <= tol2 * h_b2[q]) {
                    h_status[q] = CG_CONVERGED;
                } else {
                    h_mode[q] = 2;  // restart the recurrence: p = r
                    h_rho[q] = rt;
                    h_rho_ru[q] = rt;
                    h_status[q] = CG_ACTIVE;
                }
            }
        }
        // rho, status, iters (unchanged), ru_flag, rho_ru, true_res2, the
        // restart coefficients and modes in one copy
        HISQ_TRY(h2d(dev.rho, h_rho, state_bytes));
        if (half) HISQ_TRY(half_p_restart(vh, nrhs, ps, rs, d_rbeta, d_mode, s));
        else HISQ_TRY(mixed_p_restart(ps, rs, n, nrhs, d_rbeta, d_mode, s));
        mirror_current = true;
    }

    // fold any remaining FP32 correction into x; b = 0 gives x = 0
    HISQ_TRY(mixed_accum_x(x, xs, n, nrhs, nullptr, s));
    HISQ_TRY(d2h(h_status, dev.status, in_));
    HISQ_TRY(d2h(h_iters, dev.iters, in_));
    HISQ_TRY(d2h(h_tr2, dev.true_res2, dn));
    HISQ_TRY(sync());
    bool need_final = false;
    for (int q = 0; q < nrhs; ++q) {
        if (h_b2[q] == 0.0) HISQ_HIP(hipMemsetAsync(x + (size_t)q * n, 0, sizeof(double2) * n, s));
        need_final |= h_status[q] != CG_CONVERGED;
    }
    if (need_final) {
        HISQ_TRY(true_residual(nullptr, nullptr));
        for (int q = 0; q < nrhs; ++q)
            if (h_status[q] != CG_CONVERGED) h_tr2[q] = h_rho_t[q];
    }
    hisq_status ret = HISQ_OK;
    std::string why;
    for (int q = 0; q < nrhs; ++q) {
        const int st = h_status[q];
        if (stats) {
            hisq_cg_stats &S = stats[q];
            S.iterations = h_iters[q];
            S.true_residual_checks = ru_count[q];
            S.converged = st == CG_CONVERGED;
            S.reliable_updates = ru_count[q];
            S.redeflations = defl_count[q];
            S.reserved0 = 0;
            S.b_norm = std::sqrt(h_b2[q]);
            S.true_residual = h_b2[q] > 0.0 ? std::sqrt(h_tr2[q] / h_b2[q]) : 0.0;
        }
        if (st == CG_NAN) {
            ret = HISQ_ERR_NAN;
            why = "NaN or Inf in a CG reduction (rhs " + std::to_string(q) + ")";
        } else if (st == CG_BREAKDOWN && ret != HISQ_ERR_NAN) {
            ret = HISQ_ERR_BREAKDOWN;
            why = "<p, A p> <= 0 (rhs " + std::to_string(q) + ")";
        } else if (st != CG_CONVERGED && ret == HISQ_OK) {
            ret = HISQ_ERR_NOT_CONVERGED;
            why = "rhs " + std::to_string(q) + " did not reach tol within max_iter";
        }
    }
    if (ret != HISQ_OK) return fail(ret, why);
    return HISQ_OK;
}

}  // namespace hisq
