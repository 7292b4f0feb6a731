// hisq_cg_solve: even-odd preconditioned CG on A = (2m)^2 - D_eo D_oe for a
// batch of right-hand sides (arXiv:2502.00152, section 2: the conventional
// "CG" baseline, solved on the normal equation Eq. (1) with a true-residual
// stopping criterion).
//
// One iteration is five stream-ordered launches:
//   1. t  = D_oe p                          (half stencil, odd output)
//   2. Ap = (2m)^2 p - D_eo t, partials of Re<p, Ap>   (half stencil)
//   3. alpha = rho / Re<p, Ap>; r -= alpha Ap, partials of <r, r>
//   4. rho' = <r, r>, beta = rho' / rho, convergence state  (one wave per RHS)
//   5. x += alpha p, p = r + beta p         (old p in both)
// Scalars never leave the device.  The host polls the per-RHS state every
// check_interval iterations; a right-hand side whose iterated residual has
// crossed the tolerance is frozen until the host runs the true-residual check
// (one more application of A), which either accepts it or restarts its
// recurrence from the true residual.
#include <cmath>
#include <vector>

#include "hisq_internal.h"

namespace hisq {
hisq_status check_gauge(hisq_gauge g);
hisq_status check_vec(const void *p, const char *name);
hisq_status check_nrhs(int nrhs);
hisq_status check_mass(double two_m, bool positive);
}  // namespace hisq

using namespace hisq;

namespace {

struct CgBuffers {
    double2 *r, *p, *Ap;
    CgDev dev;
    Reduce red;
    Reduce pap;         // <p, Ap> partials of the stencil kernel
    int *host_status;   // pinned
    int *host_iters;
    int *host_checks;
    int *host_skip;     // pinned: 0 = compute A x for this RHS
    int *dev_skip;
    double *host_tr2;
    double *host_b2;
};

hisq_status alloc_cg(hisq_gauge_s *g, int nrhs, CgBuffers &B) {
    const size_t vec = sizeof(double2) * 3 * (size_t)g->geom.vh * nrhs;
    void *p = nullptr;
    HISQ_TRY(g->ws.get("cg_r", vec, &p));
    B.r = static_cast<double2 *>(p);
    HISQ_TRY(g->ws.get("cg_p", vec, &p));
    B.p = static_cast<double2 *>(p);
    HISQ_TRY(g->ws.get("cg_Ap", vec, &p));
    B.Ap = static_cast<double2 *>(p);
    // scalars: 10 double arrays + 5 int arrays of nrhs
    HISQ_TRY(g->ws.get("cg_scalars", (10 * sizeof(double) + 5 * sizeof(int)) * nrhs + 64, &p));
    double *d = static_cast<double *>(p);
    B.dev.rho = d;
    B.dev.rho_pend = d + nrhs;
    B.dev.alpha = d + 2 * nrhs;
    B.dev.beta = d + 3 * nrhs;
    B.dev.bnorm2 = d + 4 * nrhs;
    B.dev.tol2b = d + 5 * nrhs;
    B.dev.true_res2 = d + 6 * nrhs;
    B.dev.xp_alpha = d + 7 * nrhs;
    B.dev.xp_beta = d + 8 * nrhs;
    B.dev.rho_ru = d + 9 * nrhs;
    B.dev.ru_flag = nullptr;
    B.dev.delta2 = 0.0;
    B.dev.ru_freeze = 0;
    int *iv = reinterpret_cast<int *>(d + 10 * nrhs);
    B.dev.status = iv;
    B.dev.iters = iv + nrhs;
    B.dev.checks = iv + 2 * nrhs;
    B.dev.xp_mode = iv + 3 * nrhs;
    B.dev_skip = iv + 4 * nrhs;
    const int64_t n = 3 * (int64_t)g->geom.vh;
    const size_t nparts = std::max<size_t>((size_t)nrhs * dslash_reduce_blocks(g, nrhs),
                                           (size_t)2 * nrhs * blas_reduce_blocks(n));
    HISQ_TRY(g->ws.get("reduce_partials", sizeof(double) * nparts, &p));
    B.red.partials = static_cast<double *>(p);
    HISQ_TRY(g->ws.get("cg_pap_partials",
                       sizeof(double) * (size_t)nrhs * dslash_reduce_blocks(g, nrhs), &p));
    B.pap.partials = static_cast<double *>(p);
    return HISQ_OK;
}

struct PinnedHost {
    void *ptr = nullptr;
    ~PinnedHost() {
        if (ptr) (void)hipHostFree(ptr);
    }
};

}  // namespace

extern "C" hisq_status hisq_cg_solve(hisq_gauge g, double two_m, const void *b_e_dev,
                                     void *x_e_dev, int nrhs, const hisq_cg_params *params,
                                     hisq_cg_stats *stats_host, void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    if (!params) return fail(HISQ_ERR_INVALID_ARG, "params is null");
    if (params->two_m_rhs) {
        for (int q = 0; q < nrhs; ++q) HISQ_TRY(check_mass(params->two_m_rhs[q], true));
        if (params->n_ev != 0 || params->tol_restart != 0.0)
            return fail(HISQ_ERR_INVALID_ARG, "per-RHS masses do not combine with re-deflation");
        two_m = params->two_m_rhs[0];
    } else {
        HISQ_TRY(check_mass(two_m, true));
    }
    HISQ_TRY(check_vec(b_e_dev, "b_e_dev"));
    HISQ_TRY(check_vec(x_e_dev, "x_e_dev"));
    if (b_e_dev == x_e_dev) return fail(HISQ_ERR_INVALID_ARG, "b and x must not overlap");
    if (!(params->tol > 0.0) || !std::isfinite(params->tol))
        return fail(HISQ_ERR_INVALID_ARG, "tol must be finite and > 0");
    if (params->max_iter < 0) return fail(HISQ_ERR_INVALID_ARG, "max_iter must be >= 0");
    if (params->check_interval < 0) return fail(HISQ_ERR_INVALID_ARG, "check_interval < 0");
    for (int k = 0; k < 7; ++k)
        if (params->reserved[k]) return fail(HISQ_ERR_INVALID_ARG, "reserved fields must be 0");
    if (params->parity != 0 && params->parity != 1)
        return fail(HISQ_ERR_INVALID_ARG, "parity must be 0 (even) or 1 (odd)");
    if (params->parity == 1 && (params->n_ev != 0 || params->tol_restart != 0.0))
        return fail(HISQ_ERR_INVALID_ARG, "re-deflation uses even eigenvectors: parity must be 0");
    const hipStream_t caller = static_cast<hipStream_t>(stream);
    hipStream_t s = nullptr;
    HISQ_TRY(solver_stream(g, caller, &s));
    struct Rejoin {  // order the caller's stream after everything enqueued here
        hisq_gauge_s *g;
        hipStream_t c;
        ~Rejoin() { (void)solver_stream_done(g, c); }
    } rejoin{g, caller};
    const double2 *b = static_cast<const double2 *>(b_e_dev);
    double2 *x = static_cast<double2 *>(x_e_dev);
    const double *m2_rhs = nullptr;  // (2m)^2 per RHS on the device, if given
    if (params->two_m_rhs) {
        std::vector<double> m2(nrhs);
        for (int q = 0; q < nrhs; ++q) m2[q] = params->two_m_rhs[q] * params->two_m_rhs[q];
        void *pm = nullptr;
        HISQ_TRY(g->ws.get("cg_m2", sizeof(double) * nrhs, &pm));
        HISQ_HIP(hipMemcpyAsync(pm, m2.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
        HISQ_HIP(hipStreamSynchronize(s));  // m2 is a local array
        m2_rhs = static_cast<const double *>(pm);
    }
    if (params->sloppy_prec == HISQ_FP32 || params->sloppy_prec == HISQ_BF16 ||
        params->sloppy_prec == HISQ_Q16 || params->sloppy_prec == HISQ_HALF)
        return solve_mixed(g, two_m, b, x, nrhs, params, stats_host, s, m2_rhs,
                           params->sloppy_prec);
    if (params->sloppy_prec != HISQ_FP64) return fail(HISQ_ERR_INVALID_ARG, "unknown sloppy_prec");
    if (params->n_ev != 0 || params->tol_restart != 0.0)
        return fail(HISQ_ERR_INVALID_ARG,
                    "re-deflation runs at reliable updates: it needs a mixed-precision "
                    "sloppy_prec");

    const int64_t n = 3 * (int64_t)g->geom.vh;
    const int interval = params->check_interval > 0 ? params->check_interval : 16;
    const int par = params->parity;

    CgBuffers B{};
    HISQ_TRY(alloc_cg(g, nrhs, B));
    B.dev.max_iter = params->max_iter;

    // pinned host mirror of the per-RHS state
    PinnedHost pin;
    const size_t host_bytes = (4 * sizeof(int) + 2 * sizeof(double)) * nrhs + 64;
    HISQ_HIP(hipHostMalloc(&pin.ptr, host_bytes, hipHostMallocDefault));
    double *hd = static_cast<double *>(pin.ptr);
    B.host_tr2 = hd;
    B.host_b2 = hd + nrhs;
    B.host_status = reinterpret_cast<int *>(hd + 2 * nrhs);
    B.host_iters = B.host_status + nrhs;
    B.host_checks = B.host_iters + nrhs;
    B.host_skip = B.host_checks + nrhs;

    auto fetch_state = [&]() -> hisq_status {
        HISQ_HIP(hipMemcpyAsync(B.host_status, B.dev.status, 3 * sizeof(int) * nrhs,
                                hipMemcpyDeviceToHost, s));
        HISQ_HIP(hipStreamSynchronize(s));
        return HISQ_OK;
    };

    // r = b - A x0, p = r, rho = <r, r>, ||b||
    HISQ_TRY(apply_mdagm(g, two_m, x, B.Ap, nrhs, s, par, m2_rhs));
    HISQ_TRY(cg_init(n, nrhs, b, B.Ap, B.r, B.p, params->tol, B.dev, B.red, s));
    HISQ_TRY(fetch_state());

    auto count = [&](int st) {
        int c = 0;
        for (int i = 0; i < nrhs; ++i) c += B.host_status[i] == st;
        return c;
    };

    void *tmpv = nullptr;
    HISQ_TRY(g->ws.get("mdagm_tmp", sizeof(double2) * (size_t)n * nrhs, &tmpv));
    double2 *t = static_cast<double2 *>(tmpv);
    const double m2 = two_m * two_m;
    const int nb_pap = dslash_reduce_blocks(g, nrhs);
    double *pq_sum = nullptr;
    if (nb_pap >= kPapPresum) {
        void *pp = nullptr;
        HISQ_TRY(g->ws.get("cg_pq", sizeof(double) * nrhs, &pp));
        pq_sum = static_cast<double *>(pp);
    }

    auto iterate = [&]() -> hisq_status {
        HISQ_TRY(launch_dslash(g, 1 - par, B.p, t, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE,
                               &B.dev, nullptr, s));
        HISQ_TRY(launch_dslash(g, par, t, B.Ap, nrhs, B.p, m2, nullptr, 0.0, -1.0, FIN_CG_ALPHA,
                               &B.dev, &B.pap, s, m2_rhs));
        const double *pq = B.pap.partials;
        int nbq = nb_pap;
        if (pq_sum) {
            HISQ_TRY(cg_sum_pap(nrhs, B.pap.partials, nb_pap, pq_sum, s));
            pq = pq_sum;
            nbq = 1;
        }
        HISQ_TRY(cg_update_r(n, nrhs, B.r, B.Ap, pq, nbq, B.dev, B.red, s));
        HISQ_TRY(cg_finalize(n, nrhs, pq, nbq, B.dev, B.red, s));
        HISQ_TRY(cg_update_xp(n, nrhs, x, B.r, B.p, B.dev, s));
        return HISQ_OK;
    };

    // Every iteration advances each active RHS towards max_iter, and a pending
    // one is resolved at the next poll, so the loop ends; the cap below only
    // guards against a device state that never changes.
    const int64_t cap = 4 * (int64_t)params->max_iter + 4 * (int64_t)interval + 16;
    int64_t enqueued = 0;
    const bool graphs = cg_use_graphs(g, nrhs);
    GraphChunk chunk;
    const std::function<hisq_status()> chunk_body = [&]() -> hisq_status {
        for (int k = 0; k < interval; ++k) HISQ_TRY(iterate());
        return HISQ_OK;
    };
    for (;;) {
        if (count(CG_PENDING) > 0) {
            // A x for the groups holding a pending RHS only
            for (int i = 0; i < nrhs; ++i) B.host_skip[i] = B.host_status[i] == CG_PENDING ? 0 : 1;
            HISQ_HIP(hipMemcpyAsync(B.dev_skip, B.host_skip, sizeof(int) * nrhs,
                                    hipMemcpyHostToDevice, s));
            HISQ_TRY(apply_mdagm(g, two_m, x, B.Ap, nrhs, s, par, m2_rhs, B.dev_skip));
            HISQ_TRY(cg_true_residual(n, nrhs, b, B.Ap, B.r, B.dev, B.red, false, s));
            HISQ_TRY(cg_restart_p(n, nrhs, B.r, B.p, B.dev, s));
            HISQ_TRY(fetch_state());
            continue;
        }
        if (count(CG_ACTIVE) + count(CG_RESTART) == 0) break;
        if (params->max_iter == 0 || enqueued >= cap) break;
        if (t_chunk_group && enqueued > 0) {
            // with the other systems' chunks in one graph (the first chunk runs
            // eagerly, so that lazily made copies exist before any capture)
            HISQ_TRY(t_chunk_group->run(s, t_chunk_sys, chunk_body));
        } else if (graphs) {
            HISQ_TRY(chunk.run(s, chunk_body));
        } else {
            HISQ_TRY(chunk_body());
        }
        enqueued += interval;
        HISQ_TRY(fetch_state());
    }

    // b = 0 gives x = 0
    HISQ_HIP(hipMemcpyAsync(B.host_tr2, B.dev.true_res2, sizeof(double) * nrhs,
                            hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipMemcpyAsync(B.host_b2, B.dev.bnorm2, sizeof(double) * nrhs,
                            hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nrhs; ++i)
        if (B.host_b2[i] == 0.0)
            HISQ_HIP(hipMemsetAsync(x + (size_t)i * n, 0, sizeof(double2) * n, s));

    // final true residual of the right-hand sides that did not converge
    bool need_final = false;
    for (int i = 0; i < nrhs; ++i) need_final |= B.host_status[i] != CG_CONVERGED;
    if (need_final) {
        HISQ_TRY(apply_mdagm(g, two_m, x, B.Ap, nrhs, s, par, m2_rhs));
        HISQ_TRY(cg_true_residual(n, nrhs, b, B.Ap, B.r, B.dev, B.red, true, s));
        HISQ_HIP(hipMemcpyAsync(B.host_tr2, B.dev.true_res2, sizeof(double) * nrhs,
                                hipMemcpyDeviceToHost, s));
        HISQ_HIP(hipStreamSynchronize(s));
    }

    hisq_status ret = HISQ_OK;
    std::string why;
    for (int i = 0; i < nrhs; ++i) {
        const int st = B.host_status[i];
        if (stats_host) {
            hisq_cg_stats &S = stats_host[i];
            S.iterations = B.host_iters[i];
            S.true_residual_checks = B.host_checks[i];
            S.converged = st == CG_CONVERGED;
            S.reliable_updates = 0;
            S.redeflations = 0;
            S.reserved0 = 0;
            S.b_norm = std::sqrt(B.host_b2[i]);
            S.true_residual = B.host_b2[i] > 0.0 ? std::sqrt(B.host_tr2[i] / B.host_b2[i]) : 0.0;
        }
        if (st == CG_NAN) {
            ret = HISQ_ERR_NAN;
            why = "NaN or Inf in a CG reduction (rhs " + std::to_string(i) + ")";
        } else if (st == CG_BREAKDOWN && ret != HISQ_ERR_NAN) {
            ret = HISQ_ERR_BREAKDOWN;
            why = "<p, A p> <= 0 (rhs " + std::to_string(i) + ")";
        } else if (st != CG_CONVERGED && ret == HISQ_OK) {
            ret = HISQ_ERR_NOT_CONVERGED;
            why = "rhs " + std::to_string(i) + " did not reach tol within max_iter";
        }
    }
    if (ret != HISQ_OK) return fail(ret, why);
    return HISQ_OK;
}
