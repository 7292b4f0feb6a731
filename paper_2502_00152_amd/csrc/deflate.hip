// hisq_deflate: the deflation initial guess of arXiv:2502.00152, Eq. (4),
//   x0 = sum_i v_i (1 / lambda_i) v_i^H b,  lambda_i = eps_i + (2m)^2
// (Eq. (3): the massive eigenvalue is the massless one shifted by (2m)^2; the
// eigenvectors do not depend on the mass).  Two contractions on the FP64
// matrix cores: c = diag(1/lambda) V^H B, then X0 = V c.  The eigenvectors may
// be stored in FP32 (section 3: single-precision eigenvectors).
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

extern "C" hisq_status hisq_deflate(hisq_gauge g, int n_ev, const void *evecs_dev,
                                    hisq_prec evec_prec, const double *evals_host, double two_m,
                                    const void *b_e_dev, void *x0_e_dev, int nrhs, void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_mass(two_m, false));
    const int64_t N = 3 * (int64_t)g->geom.vh;
    if (n_ev < 1 || n_ev > N) return fail(HISQ_ERR_INVALID_ARG, "n_ev must be in [1, 3*Vh]");
    if (!evals_host) return fail(HISQ_ERR_INVALID_ARG, "evals_host is null");
    if (evec_prec != HISQ_FP64 && evec_prec != HISQ_FP32)
        return fail(HISQ_ERR_INVALID_ARG, "evec_prec must be HISQ_FP64 or HISQ_FP32");
    HISQ_TRY(check_vec(evecs_dev, "evecs_dev"));
    HISQ_TRY(check_vec(b_e_dev, "b_e_dev"));
    HISQ_TRY(check_vec(x0_e_dev, "x0_e_dev"));
    if (x0_e_dev == b_e_dev || x0_e_dev == evecs_dev)
        return fail(HISQ_ERR_INVALID_ARG, "x0 must not overlap b or the eigenvectors");
    std::vector<double> w(n_ev);
    const double m2 = two_m * two_m;
    for (int i = 0; i < n_ev; ++i) {
        const double lam = evals_host[i] + m2;
        if (!std::isfinite(lam) || !(lam > 0.0))
            return fail(HISQ_ERR_INVALID_ARG, "eps_i + (2m)^2 must be finite and > 0");
        w[i] = 1.0 / lam;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *wd = nullptr, *cd = nullptr;
    HISQ_TRY(g->ws.get("deflate_w", sizeof(double) * n_ev, &wd));
    HISQ_TRY(g->ws.get("deflate_c", sizeof(double2) * (size_t)n_ev * nrhs, &cd));
    // pageable source: the copy has consumed w when the call returns
    HISQ_HIP(hipMemcpyAsync(wd, w.data(), sizeof(double) * n_ev, hipMemcpyHostToDevice, s));
    double2 *C = static_cast<double2 *>(cd);
    const double2 *B = static_cast<const double2 *>(b_e_dev);
    double2 *X = static_cast<double2 *>(x0_e_dev);
    if (evec_prec == HISQ_FP32) {
        const float2 *V = static_cast<const float2 *>(evecs_dev);
        HISQ_TRY(gemm_tn(g, V, n_ev, B, nrhs, N, static_cast<const double *>(wd), 1.0, C, s));
        HISQ_TRY(gemm_nn(V, n_ev, C, nrhs, N, 0.0, X, s));
    } else {
        const double2 *V = static_cast<const double2 *>(evecs_dev);
        HISQ_TRY(gemm_tn(g, V, n_ev, B, nrhs, N, static_cast<const double *>(wd), 1.0, C, s));
        HISQ_TRY(gemm_nn(V, n_ev, C, nrhs, N, 0.0, X, s));
    }
    return HISQ_OK;
}
