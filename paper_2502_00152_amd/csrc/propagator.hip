// hisq_propagator_solve: the whole solve of M psi = eta for full-lattice
// sources (arXiv:2502.00152, section 2: even-odd preconditioning, the even
// solve, reconstruction of the odd sites and the CG polish of the odd
// solution, as in the MILC + QUDA workflow the paper describes).
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

extern "C" hisq_status hisq_propagator_solve(hisq_gauge g, double two_m, const void *eta_dev,
                                             void *psi_dev, int nrhs,
                                             const hisq_prop_params *params,
                                             hisq_prop_stats *stats_host, void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_mass(two_m, true));
    HISQ_TRY(check_vec(eta_dev, "eta_dev"));
    HISQ_TRY(check_vec(psi_dev, "psi_dev"));
    if (!params) return fail(HISQ_ERR_INVALID_ARG, "params is null");
    for (int k = 0; k < 7; ++k)
        if (params->reserved[k]) return fail(HISQ_ERR_INVALID_ARG, "reserved fields must be 0");
    if (params->cg.parity != 0) return fail(HISQ_ERR_INVALID_ARG, "cg.parity must be 0");
    if (params->polish_tol < 0.0 || !std::isfinite(params->polish_tol))
        return fail(HISQ_ERR_INVALID_ARG, "polish_tol must be finite and >= 0");
    if (params->polish_max_iter < 0) return fail(HISQ_ERR_INVALID_ARG, "polish_max_iter < 0");
    const int64_t n = 3 * (int64_t)g->geom.vh;
    const size_t full_bytes = sizeof(double2) * 2 * (size_t)n * nrhs;
    {
        const char *a = static_cast<const char *>(eta_dev), *b = static_cast<const char *>(psi_dev);
        if (a < b + full_bytes && b < a + full_bytes)
            return fail(HISQ_ERR_INVALID_ARG, "eta and psi must not overlap");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t vb = sizeof(double2) * (size_t)n * nrhs;
    double2 *ee, *eo, *y, *xe, *xo, *t;
    void *p = nullptr;
    HISQ_TRY(g->ws.get("prop_eta_e", vb, &p));
    ee = static_cast<double2 *>(p);
    HISQ_TRY(g->ws.get("prop_eta_o", vb, &p));
    eo = static_cast<double2 *>(p);
    HISQ_TRY(g->ws.get("prop_y", vb, &p));
    y = static_cast<double2 *>(p);
    HISQ_TRY(g->ws.get("prop_psi_e", vb, &p));
    xe = static_cast<double2 *>(p);
    HISQ_TRY(g->ws.get("prop_psi_o", vb, &p));
    xo = static_cast<double2 *>(p);
    HISQ_TRY(g->ws.get("prop_tmp", vb, &p));
    t = static_cast<double2 *>(p);

    std::vector<hisq_cg_stats> se(nrhs), sp(nrhs);
    // eta -> (eta_e, eta_o);  y_e = 2m eta_e - D_eo eta_o
    HISQ_TRY(launch_split(g, static_cast<const double2 *>(eta_dev), ee, eo, nrhs, s));
    HISQ_TRY(launch_dslash(g, 0, eo, y, nrhs, ee, two_m, nullptr, 0.0, -1.0, FIN_NONE, nullptr,
                           nullptr, s));
    // initial guess: zero, or the deflation guess of Eq. (4)
    const hisq_cg_params &cg = params->cg;
    if (cg.n_ev > 0) {
        HISQ_TRY(hisq_deflate(g, cg.n_ev, cg.evecs_dev, cg.evec_prec, cg.evals_host, two_m, y, xe,
                              nrhs, stream));
    } else {
        HISQ_HIP(hipMemsetAsync(xe, 0, vb, s));
    }
    const hisq_status st_even = hisq_cg_solve(g, two_m, y, xe, nrhs, &cg, se.data(), stream);
    if (st_even != HISQ_OK && st_even != HISQ_ERR_NOT_CONVERGED) return st_even;
    const std::string why_even = st_even == HISQ_OK ? std::string() : hisq_last_error();
    // psi_o = (eta_o - D_oe psi_e) / (2m)
    const double inv = 1.0 / two_m;
    HISQ_TRY(launch_dslash(g, 1, xe, xo, nrhs, eo, inv, nullptr, 0.0, -inv, FIN_NONE, nullptr,
                           nullptr, s));
    hisq_status st_pol = HISQ_OK;
    std::string why_pol;
    if (params->polish_tol > 0.0) {
        // y_o = 2m eta_o - D_oe eta_e = (M^H eta)_o; CG on (M^H M)_oo from psi_o
        HISQ_TRY(launch_dslash(g, 1, ee, y, nrhs, eo, two_m, nullptr, 0.0, -1.0, FIN_NONE, nullptr,
                               nullptr, s));
        hisq_cg_params pp = cg;
        pp.tol = params->polish_tol;
        if (params->polish_max_iter > 0) pp.max_iter = params->polish_max_iter;
        pp.parity = 1;
        pp.n_ev = 0;
        pp.evecs_dev = nullptr;
        pp.evals_host = nullptr;
        pp.tol_restart = 0.0;
        st_pol = hisq_cg_solve(g, two_m, y, xo, nrhs, &pp, sp.data(), stream);
        if (st_pol != HISQ_OK && st_pol != HISQ_ERR_NOT_CONVERGED) return st_pol;
        if (st_pol != HISQ_OK) why_pol = hisq_last_error();
    }
    HISQ_TRY(launch_merge(g, xe, xo, static_cast<double2 *>(psi_dev), nrhs, s));

    // residual of M psi = eta: even rows 2m psi_e + D_eo psi_o, odd rows
    // 2m psi_o + D_oe psi_e, each against eta (y, no longer needed, takes the
    // residual vectors)
    Reduce red{};
    HISQ_TRY(g->ws.get("reduce_partials", sizeof(double) * (size_t)nrhs * mixed_resid_blocks(n), &p));
    red.partials = static_cast<double *>(p);
    HISQ_TRY(g->ws.get("prop_norms", sizeof(double) * 4 * (size_t)nrhs, &p));
    double *d_norms = static_cast<double *>(p);
    HISQ_TRY(g->ws.get("prop_zero", vb, &p));
    double2 *zero = static_cast<double2 *>(p);
    HISQ_HIP(hipMemsetAsync(zero, 0, vb, s));
    HISQ_TRY(launch_dslash(g, 0, xo, t, nrhs, xe, two_m, nullptr, 0.0, 1.0, FIN_NONE, nullptr,
                           nullptr, s));
    HISQ_TRY(mixed_resid(ee, t, y, n, nrhs, nullptr, d_norms, red, s));
    HISQ_TRY(launch_dslash(g, 1, xe, t, nrhs, xo, two_m, nullptr, 0.0, 1.0, FIN_NONE, nullptr,
                           nullptr, s));
    HISQ_TRY(mixed_resid(eo, t, y, n, nrhs, nullptr, d_norms + nrhs, red, s));
    HISQ_TRY(mixed_resid(ee, zero, y, n, nrhs, nullptr, d_norms + 2 * nrhs, red, s));
    HISQ_TRY(mixed_resid(eo, zero, y, n, nrhs, nullptr, d_norms + 3 * nrhs, red, s));
    std::vector<double> h(4 * (size_t)nrhs);
    HISQ_HIP(hipMemcpyAsync(h.data(), d_norms, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    if (stats_host) {
        for (int q = 0; q < nrhs; ++q) {
            hisq_prop_stats &S = stats_host[q];
            S = hisq_prop_stats{};
            S.even = se[q];
            if (params->polish_tol > 0.0) S.polish = sp[q];
            const double e2 = h[2 * nrhs + q] + h[3 * nrhs + q];
            S.residual = e2 > 0.0 ? std::sqrt((h[q] + h[nrhs + q]) / e2) : 0.0;
            S.residual_even = e2 > 0.0 ? std::sqrt(h[q] / e2) : 0.0;
        }
    }
    if (st_even != HISQ_OK) return fail(st_even, "even solve: " + why_even);
    if (st_pol != HISQ_OK) return fail(st_pol, "odd polish: " + why_pol);
    return HISQ_OK;
}
