// hisq_eigensolve: lowest eigenpairs of A = (2m)^2 - D_eo D_oe on even sites by
// thick-restart Lanczos on a Chebyshev-filtered A, closed by a Rayleigh-Ritz
// step on A itself (arXiv:2502.00152, section 2: eigenvectors of the squared
// operator from thick-restart Lanczos, used for deflation; section 3:
// single-parity vectors).
//
// Outline
//   1. Pilot: plain Lanczos on A (full re-orthogonalisation, n_kr steps) gives
//      an upper bound b of the spectrum and a cut a above the wanted part.  By
//      Cauchy interlacing the (n_ev+1)-th smallest Ritz value is at least the
//      (n_ev+1)-th eigenvalue, so at least n_ev eigenvalues lie below a.
//   2. Filter p(A) = T_d(l(A)), l(x) = (a + b - 2x) / (b - a): eigenvalues in
//      [a, b] map into [-1, 1], those below a above 1, monotonically, so the
//      largest eigenvalues of p(A) belong to the smallest of A.
//   3. Thick-restart Lanczos on p(A) with classical Gram-Schmidt applied twice
//      against the whole basis; after each cycle the small arrowhead +
//      tridiagonal matrix is diagonalised on the host, the Ritz vectors of
//      the kept part become the new leading basis and the residual vector the
//      next one.
//   4. When the n_ev wanted Ritz values have residuals below tol (relative to
//      each Ritz value), form the Ritz vectors, apply A to them, diagonalise
//      the Gram matrix U^H A U on the host, rotate, and accept when every
//      ||A v - lambda v|| <= tol * lambda_max; otherwise tighten and go on.
//
// Memory: one FP64 basis of n_kr + 1 vectors.  Basis rotations V <- V Y are
// done in place, block of rows by block of rows through a scratch block (each
// row of the result depends only on the same row of V); A U for the Gram
// matrix and the residuals is formed a block of columns at a time.  All
// buffers are freed before the call returns.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "hisq_internal.h"

namespace hisq {
hisq_status check_gauge(hisq_gauge g);
hisq_status check_vec(const void *p, const char *name);
hisq_status check_mass(double two_m, bool positive);
int heev_jacobi(int n, std::complex<double> *A, double *w, std::complex<double> *Z, int max_sweeps);
int syev_qr(int n, double *A, double *w, double *Z);
hisq_status vec_random(double2 *x, int64_t n, uint64_t seed, hipStream_t s);
hisq_status vec_dot(hisq_gauge_s *g, const double2 *x, const double2 *y, int64_t n, double *out,
                    hipStream_t s);
hisq_status vec_axpby2(double2 *y, double a, const double2 *x1, double b1, const double2 *x2,
                       double b2, int64_t n, hipStream_t s);
hisq_status vec_col_residuals(hisq_gauge_s *g, const double2 *W, const double2 *U,
                              const double *lam_dev, int64_t n, int k, double *out_dev,
                              hipStream_t s);
}  // namespace hisq

constexpr const char *const kEigBuffers[] = {"eig_V", "eig_T", "eig_w", "eig_y1", "eig_y2",
                                             "eig_coef", "eig_scal"};

using namespace hisq;
using cd = std::complex<double>;

namespace {

struct Pinned {
    void *ptr = nullptr;
    ~Pinned() {
        if (ptr) (void)hipHostFree(ptr);
    }
};

class Solver {
public:
    Solver(hisq_gauge_s *g, double two_m, hipStream_t s)
        : g_(g), two_m_(two_m), s_(s), N_(3 * (int64_t)g->geom.vh) {}

    hisq_gauge_s *g_;
    double two_m_;
    hipStream_t s_;
    int64_t N_;
    double2 *V_ = nullptr;     // the basis: cols_ columns of N_
    double2 *T_ = nullptr;     // scratch: tcols_ columns of N_ (row blocks of rotations,
                               // blocks of A U)
    double2 *w_ = nullptr, *y1_ = nullptr, *y2_ = nullptr;
    double2 *coef_ = nullptr;  // device complex coefficients (GEMM operands)
    double *dscal_ = nullptr;  // device scalars
    double *hscal_ = nullptr;  // pinned host mirror
    Pinned pin_;
    int matvecs_ = 0;
    int gs_passes_ = 0;  // Gram-Schmidt passes (for the statistics)
    int nkr_ = 0;
    int cols_ = 0;         // columns of the basis buffer
    int tcols_ = 0;        // columns of the scratch block
    int64_t rows_blk_ = 0; // rows per block of an in-place rotation
    bool bad_col_ = false; // a column index outside [0, cols_) was requested
    size_t coef_cap_ = 0;

    // Column i of the basis; an index outside the allocation is a
    // programming error: it is recorded and the first column returned instead.
    double2 *col(double2 *base, int i, int count = 1) {
        const int lim = base == T_ ? tcols_ : cols_;
        if (i < 0 || count < 1 || i + count > lim) {
            bad_col_ = true;
            return base;
        }
        return base + (size_t)i * N_;
    }
    hisq_status check_cols() const {
        return bad_col_ ? fail(HISQ_ERR_INVALID_ARG, "eigensolve: basis column out of range")
                        : HISQ_OK;
    }

    hisq_status alloc(int nkr, int n_ev) {
        nkr_ = nkr;
        void *p = nullptr;
        const size_t vb = sizeof(double2) * (size_t)N_;
        cols_ = nkr + 1;
        tcols_ = std::min(n_ev, 32);
        // rows of one block of an in-place rotation of up to nkr columns
        rows_blk_ = std::max<int64_t>(8, (int64_t)tcols_ * N_ / nkr / 8 * 8);
        rows_blk_ = std::min<int64_t>(rows_blk_, N_);
        HISQ_TRY(g_->ws.get("eig_V", vb * cols_, &p));
        V_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_T", std::max(vb * tcols_, sizeof(double2) * (size_t)rows_blk_ * nkr),
                            &p));
        T_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_w", vb, &p));
        w_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_y1", vb, &p));
        y1_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_y2", vb, &p));
        y2_ = static_cast<double2 *>(p);
        coef_cap_ = (size_t)(nkr + 1) * std::max(nkr + 1, n_ev) + 64;
        HISQ_TRY(g_->ws.get("eig_coef", sizeof(double2) * coef_cap_, &p));
        coef_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_scal", sizeof(double) * (4 + 2 * (size_t)n_ev), &p));
        dscal_ = static_cast<double *>(p);
        HISQ_HIP(hipHostMalloc(&pin_.ptr, sizeof(double) * (4 + 2 * (size_t)n_ev),
                               hipHostMallocDefault));
        hscal_ = static_cast<double *>(pin_.ptr);
        return HISQ_OK;
    }

    void release() {
        (void)hipStreamSynchronize(s_);
        for (const char *b : kEigBuffers) g_->ws.release_one(b);
    }

    hisq_status applyA(const double2 *in, double2 *out, int nrhs = 1) {
        matvecs_ += nrhs;
        return apply_mdagm(g_, two_m_, in, out, nrhs, s_);
    }

    hisq_status dot(const double2 *x, const double2 *y, cd *out) {
        HISQ_TRY(vec_dot(g_, x, y, N_, dscal_, s_));
        HISQ_HIP(hipMemcpyAsync(hscal_, dscal_, 2 * sizeof(double), hipMemcpyDeviceToHost, s_));
        HISQ_HIP(hipStreamSynchronize(s_));
        *out = cd(hscal_[0], hscal_[1]);
        return HISQ_OK;
    }

    hisq_status norm(const double2 *x, double *out) {
        cd d;
        HISQ_TRY(dot(x, x, &d));
        *out = std::sqrt(std::max(d.real(), 0.0));
        return HISQ_OK;
    }

    // w -= Q[0..j) (Q[0..j)^H w), twice (Q = the Lanczos basis by default)
    // Classical Gram-Schmidt against Q[0..j), repeated once when the first
    // pass removed most of w (||w'|| < ||w|| / sqrt(2), the criterion of
    // Daniel, Gragg, Kaufman and Stewart): one pass leaves w orthogonal to
    // working precision unless cancellation was large.
    hisq_status orthogonalise(double2 *w, int j, const double2 *Q = nullptr) {
        if (j <= 0) return HISQ_OK;
        if (!Q) Q = V_;
        double h0 = 0.0;
        HISQ_TRY(norm(w, &h0));
        for (int pass = 0; pass < 2; ++pass) {
            HISQ_TRY(gemm_tn(g_, Q, j, w, 1, N_, nullptr, -1.0, coef_, s_));
            HISQ_TRY(gemm_nn(Q, j, coef_, 1, N_, 1.0, w, s_));
            ++gs_passes_;
            if (pass == 0) {
                double h1 = 0.0;
                HISQ_TRY(norm(w, &h1));
                if (h1 > 0.70710678118654752 * h0) break;
            }
        }
        return HISQ_OK;
    }

    // p(x) = T_d(l(x)) for a scalar x
    static double cheb_value(double x, int d, double a, double b) {
        const double l = (a + b - 2.0 * x) / (b - a);
        if (std::fabs(l) <= 1.0) return std::cos(d * std::acos(l));
        const double v = std::cosh(d * std::acosh(std::fabs(l)));
        return (l < 0.0 && (d & 1)) ? -v : v;
    }

    // out = X Y, Y host complex [k][n] row-major (columns = new vectors): X has k columns
    hisq_status rotate(const double2 *X, int k, const std::vector<cd> &Y, int ldY, int n,
                       double2 *out) {
        // device coefficients C[j][i] = Y[i][j]
        std::vector<cd> C((size_t)n * k);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < k; ++i) C[(size_t)j * k + i] = Y[(size_t)i * ldY + j];
        if (C.size() > coef_cap_) return fail(HISQ_ERR_INVALID_ARG, "eigensolve: coefficient buffer");
        HISQ_HIP(hipMemcpyAsync(coef_, C.data(), sizeof(double2) * C.size(), hipMemcpyHostToDevice,
                                s_));
        HISQ_TRY(gemm_nn(X, k, coef_, n, N_, 0.0, out, s_));
        return HISQ_OK;
    }

    // X[:, 0:n] = X[:, 0:k] Y[0:k, 0:n] in place (n <= k; X with columns N_
    // apart), Y host complex row-major with leading dimension ldY: each block
    // of rows goes through the scratch block, which the block reads entirely
    // before its rows are overwritten.
    hisq_status rotate_inplace(double2 *X, int k, const std::vector<cd> &Y, int ldY, int n,
                               bool conj_transpose = false) {
        if (n > k || n > nkr_)
            return fail(HISQ_ERR_INVALID_ARG, "eigensolve: rotation block too large");
        std::vector<cd> C((size_t)n * k);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < k; ++i)
                C[(size_t)j * k + i] =
                    conj_transpose ? std::conj(Y[(size_t)j * ldY + i]) : Y[(size_t)i * ldY + j];
        if (C.size() > coef_cap_) return fail(HISQ_ERR_INVALID_ARG, "eigensolve: coefficient buffer");
        HISQ_HIP(hipMemcpyAsync(coef_, C.data(), sizeof(double2) * C.size(), hipMemcpyHostToDevice,
                                s_));
        for (int64_t r0 = 0; r0 < N_; r0 += rows_blk_) {
            const int64_t rows = std::min<int64_t>(rows_blk_, N_ - r0);
            HISQ_TRY(gemm_nn_ld(X + r0, N_, k, coef_, n, rows, 0.0, T_, rows, s_));
            HISQ_HIP(hipMemcpy2DAsync(X + r0, sizeof(double2) * (size_t)N_, T_,
                                      sizeof(double2) * (size_t)rows, sizeof(double2) * (size_t)rows,
                                      (size_t)n, hipMemcpyDeviceToDevice, s_));
        }
        return HISQ_OK;  // pageable source: the copy consumed C before returning
    }

    // w = T_d(l(A)) v with l(x) = (a + b - 2x) / (b - a)
    hisq_status chebyshev(const double2 *v, double2 *w, int d, double a, double b) {
        const double s1 = (a + b) / (b - a), s2 = -2.0 / (b - a);
        const double m2 = two_m_ * two_m_;
        void *tp = nullptr;
        HISQ_TRY(g_->ws.get("mdagm_tmp", sizeof(double2) * (size_t)N_, &tp));
        double2 *t = static_cast<double2 *>(tp);
        // y1 = l(A) v = (s1 + s2 m2) v - s2 D_eo D_oe v
        double2 *prev = nullptr, *cur = nullptr;
        {
            double2 *dst = d == 1 ? w : y1_;
            HISQ_TRY(launch_dslash(g_, 1, v, t, 1, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE,
                                   nullptr, nullptr, s_));
            HISQ_TRY(launch_dslash(g_, 0, t, dst, 1, v, s1 + s2 * m2, nullptr, 0.0, -s2, FIN_NONE,
                                   nullptr, nullptr, s_));
            ++matvecs_;
            prev = const_cast<double2 *>(v);
            cur = dst;
        }
        // y_{i+1} = 2 l(A) y_i - y_{i-1}
        for (int i = 1; i < d; ++i) {
            double2 *dst = (i == d - 1) ? w : (prev == v ? y2_ : prev);
            HISQ_TRY(launch_dslash(g_, 1, cur, t, 1, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE,
                                   nullptr, nullptr, s_));
            HISQ_TRY(launch_dslash(g_, 0, t, dst, 1, cur, 2.0 * (s1 + s2 * m2), prev, -1.0,
                                   -2.0 * s2, FIN_NONE, nullptr, nullptr, s_));
            ++matvecs_;
            prev = cur;
            cur = dst;
        }
        return HISQ_OK;
    }

    // After w has been orthogonalised against V[0..j]: beta = ||w||, V[j+1] = w / beta.
    // On breakdown (beta tiny) a fresh random vector orthogonal to the basis is used
    // and beta is set to 0, decoupling the new Krylov block.
    hisq_status next_vector(int j, double scale, uint64_t seed, double *beta) {
        double b = 0.0;
        HISQ_TRY(norm(w_, &b));
        if (!std::isfinite(b)) return fail(HISQ_ERR_NAN, "eigensolve: NaN in the Lanczos vector");
        if (b <= 1e-12 * scale) {
            HISQ_TRY(vec_random(w_, N_, seed, s_));
            HISQ_TRY(orthogonalise(w_, j + 1));
            double nb = 0.0;
            HISQ_TRY(norm(w_, &nb));
            if (!(nb > 0.0)) return fail(HISQ_ERR_BREAKDOWN, "eigensolve: basis exhausted");
            HISQ_TRY(vec_axpby2(col(V_, j + 1), 0.0, w_, 1.0 / nb, nullptr, 0.0, N_, s_));
            *beta = 0.0;
            return HISQ_OK;
        }
        HISQ_TRY(vec_axpby2(col(V_, j + 1), 0.0, w_, 1.0 / b, nullptr, 0.0, N_, s_));
        *beta = b;
        return HISQ_OK;
    }
};

// Eigen-decomposition of a small Hermitian matrix held as complex (row-major):
// the real symmetric Lanczos matrices go to the Householder + implicit QR
// solver (O(n^3), 0.6 s at n = 512 against 11 s for Jacobi), complex ones
// (the Rayleigh-Ritz Gram matrix) to cyclic Jacobi.
int small_heev(int n, std::vector<cd> &A, std::vector<double> &w, std::vector<cd> &Z) {
    w.assign(n, 0.0);
    Z.assign((size_t)n * n, 0.0);
    bool real = true;
    for (const cd &v : A) real = real && v.imag() == 0.0;
    if (!real) return heev_jacobi(n, A.data(), w.data(), Z.data(), 100);
    std::vector<double> Ar((size_t)n * n), Zr((size_t)n * n);
    for (size_t i = 0; i < Ar.size(); ++i) Ar[i] = A[i].real();
    const int st = syev_qr(n, Ar.data(), w.data(), Zr.data());
    for (size_t i = 0; i < Zr.size(); ++i) Z[i] = Zr[i];
    return st;
}

}  // namespace

extern "C" hisq_status hisq_eigensolve(hisq_gauge g, double two_m, int n_ev,
                                       const hisq_eig_params *params, void *evecs_dev,
                                       double *evals_host, hisq_eig_stats *stats_host,
                                       void *stream) {
    const auto t_start = std::chrono::steady_clock::now();
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_mass(two_m, false));
    HISQ_TRY(check_vec(evecs_dev, "evecs_dev"));
    if (!evals_host) return fail(HISQ_ERR_INVALID_ARG, "evals_host is null");
    if (!params) return fail(HISQ_ERR_INVALID_ARG, "params is null");
    for (int k = 0; k < 8; ++k)
        if (params->reserved[k]) return fail(HISQ_ERR_INVALID_ARG, "reserved fields must be 0");
    const int64_t N = 3 * (int64_t)g->geom.vh;
    if (n_ev < 1 || n_ev >= N) return fail(HISQ_ERR_INVALID_ARG, "n_ev must be in [1, 3*Vh)");
    int nkr = params->n_kr > 0 ? params->n_kr : std::max(2 * n_ev, n_ev + 32);
    if (params->n_kr <= 0) nkr = (int)std::min<int64_t>(nkr, N - 1);
    if (nkr <= n_ev || nkr >= N)
        return fail(HISQ_ERR_INVALID_ARG, "need n_ev < n_kr < 3*Vh");
    const double tol = params->tol > 0.0 ? params->tol : 1e-10;
    const int max_restarts = params->max_restarts > 0 ? params->max_restarts : 200;
    if (params->cheb_a < 0.0 || params->cheb_b < 0.0 || params->cheb_degree < 0)
        return fail(HISQ_ERR_INVALID_ARG, "Chebyshev parameters must be >= 0");

    const int evec_prec = params->evec_prec;
    if (evec_prec != HISQ_FP64 && evec_prec != HISQ_FP32)
        return fail(HISQ_ERR_INVALID_ARG, "evec_prec must be HISQ_FP64 or HISQ_FP32");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Solver S(g, two_m, s);
    struct Release {  // the basis and scratch are freed on every return path
        Solver &S;
        ~Release() { S.release(); }
    } release{S};
    HISQ_TRY(S.alloc(nkr, n_ev));
    const uint64_t seed = params->seed;
    auto report = [&](int restart, int step) {
        if (!params->progress) return;
        const double sec =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        params->progress(params->progress_user, restart, step, (int)S.matvecs_, sec);
    };

    // ---------------------------------------------------------------- pilot
    HISQ_TRY(vec_random(S.col(S.V_, 0), N, seed, s));
    {
        double nv = 0.0;
        HISQ_TRY(S.norm(S.col(S.V_, 0), &nv));
        HISQ_TRY(vec_axpby2(S.col(S.V_, 0), 1.0 / nv, nullptr, 0.0, nullptr, 0.0, N, s));
    }
    const int m = nkr;
    std::vector<double> al(m, 0.0), be(m, 0.0);
    double scale = 0.0;
    for (int j = 0; j < m; ++j) {
        HISQ_TRY(S.applyA(S.col(S.V_, j), S.w_));
        cd a;
        HISQ_TRY(S.dot(S.col(S.V_, j), S.w_, &a));
        al[j] = a.real();
        scale = std::max(scale, std::abs(al[j]));
        HISQ_TRY(vec_axpby2(S.w_, 1.0, S.col(S.V_, j), -al[j], j > 0 ? S.col(S.V_, j - 1) : nullptr,
                            j > 0 ? -be[j - 1] : 0.0, N, s));
        HISQ_TRY(S.orthogonalise(S.w_, j + 1));
        HISQ_TRY(S.next_vector(j, scale, seed + 1000 + j, &be[j]));
        report(-1, j);
    }
    double lam_max = 0.0, cut = 0.0;
    std::vector<cd> Vstart_coef;
    {
        std::vector<cd> T((size_t)m * m, 0.0), Z;
        std::vector<double> th;
        for (int j = 0; j < m; ++j) {
            T[(size_t)j * m + j] = al[j];
            if (j + 1 < m) T[(size_t)j * m + j + 1] = T[(size_t)(j + 1) * m + j] = be[j];
        }
        if (small_heev(m, T, th, Z) < 0)
            return fail(HISQ_ERR_BREAKDOWN, "eigensolve: pilot eigenproblem did not converge");
        const double rtop = std::abs(be[m - 1] * Z[(size_t)(m - 1) * m + (m - 1)].real()) +
                            std::abs(be[m - 1] * Z[(size_t)(m - 1) * m + (m - 1)].imag());
        lam_max = th[m - 1] + rtop;
        cut = th[std::min(n_ev, m - 1)];
        // start the filtered iteration from the sum of the lowest pilot Ritz vectors
        Vstart_coef.assign(m, 0.0);
        for (int i = 0; i < n_ev; ++i)
            for (int r = 0; r < m; ++r) Vstart_coef[r] += Z[(size_t)r * m + i];
    }
    const double b = params->cheb_b > 0.0 ? params->cheb_b : 1.02 * lam_max;
    double a = params->cheb_a > 0.0 ? params->cheb_a : cut;
    const bool auto_a = !(params->cheb_a > 0.0), auto_deg = params->cheb_degree <= 0;
    if (!(a < b)) return fail(HISQ_ERR_INVALID_ARG, "Chebyshev interval needs a < b");
    int deg = params->cheb_degree;
    if (deg <= 0) {
        const double l0 = (a + b - 2.0 * two_m * two_m) / (b - a);
        const double ac = std::acosh(std::max(l0, 1.0 + 1e-12));
        deg = (int)std::ceil(14.0 / ac);
        deg = std::max(8, std::min(deg, 120));
    }

    // ------------------------------------------------- filtered thick restart
    HISQ_TRY(S.rotate(S.V_, m, Vstart_coef, 1, 1, S.w_));
    {
        double nv = 0.0;
        HISQ_TRY(S.norm(S.w_, &nv));
        HISQ_TRY(vec_axpby2(S.col(S.V_, 0), 0.0, S.w_, 1.0 / nv, nullptr, 0.0, N, s));
    }
    std::vector<double> alpha(nkr, 0.0), beta(nkr, 0.0), theta, sigma;
    int k0 = 0, restarts = 0;
    double tol_l = tol, max_res = INFINITY;
    bool accepted = false;
    std::vector<double> lam_out(n_ev, 0.0);
    hisq_status final_status = HISQ_ERR_NOT_CONVERGED;
    double fscale = 0.0;
    int cut_updates = 0;
    for (; restarts <= max_restarts; ++restarts) {
        for (int j = k0; j < nkr; ++j) {
            HISQ_TRY(S.chebyshev(S.col(S.V_, j), S.w_, deg, a, b));
            if (j == k0 && k0 > 0) {
                // w -= sum_i sigma_i v_i
                std::vector<cd> c(k0);
                for (int i = 0; i < k0; ++i) c[i] = -sigma[i];
                HISQ_HIP(hipMemcpyAsync(S.coef_, c.data(), sizeof(double2) * k0,
                                        hipMemcpyHostToDevice, s));
                HISQ_TRY(gemm_nn(S.V_, k0, S.coef_, 1, N, 1.0, S.w_, s));
            } else if (j > k0) {
                HISQ_TRY(vec_axpby2(S.w_, 1.0, S.col(S.V_, j - 1), -beta[j - 1], nullptr, 0.0, N, s));
            }
            cd aj;
            HISQ_TRY(S.dot(S.col(S.V_, j), S.w_, &aj));
            alpha[j] = aj.real();
            fscale = std::max(fscale, std::abs(alpha[j]));
            HISQ_TRY(vec_axpby2(S.w_, 1.0, S.col(S.V_, j), -alpha[j], nullptr, 0.0, N, s));
            HISQ_TRY(S.orthogonalise(S.w_, j + 1));
            HISQ_TRY(S.next_vector(j, fscale, seed + 7777 + 131 * restarts + j, &beta[j]));
            report(restarts, j);
        }
        HISQ_TRY(S.check_cols());
        // projected matrix: arrowhead (kept Ritz values + couplings) + tridiagonal
        std::vector<cd> T((size_t)nkr * nkr, 0.0), Z;
        std::vector<double> th;
        for (int i = 0; i < k0; ++i) {
            T[(size_t)i * nkr + i] = theta[i];
            T[(size_t)i * nkr + k0] = T[(size_t)k0 * nkr + i] = sigma[i];
        }
        for (int j = k0; j < nkr; ++j) {
            T[(size_t)j * nkr + j] = alpha[j];
            if (j + 1 < nkr) T[(size_t)j * nkr + j + 1] = T[(size_t)(j + 1) * nkr + j] = beta[j];
        }
        if (small_heev(nkr, T, th, Z) < 0)
            return fail(HISQ_ERR_BREAKDOWN, "eigensolve: projected eigenproblem did not converge");
        // descending order: the largest filtered values belong to the smallest of A
        std::vector<double> Th(nkr);
        std::vector<cd> Y((size_t)nkr * nkr);
        for (int c2 = 0; c2 < nkr; ++c2) {
            Th[c2] = th[nkr - 1 - c2];
            for (int r = 0; r < nkr; ++r) Y[(size_t)r * nkr + c2] = Z[(size_t)r * nkr + (nkr - 1 - c2)];
        }
        const double bl = beta[nkr - 1];
        // Tighten the cut.  If the (kc+1)-th largest Ritz value of p(A) exceeds 1,
        // interlacing puts at least kc+1 eigenvalues of A at or below
        // p^{-1}(that value), so it is a valid cut with n_ev < kc + 1.
        if (auto_a && cut_updates < 4 && restarts < max_restarts) {
            const int kc = std::min(nkr - 1, n_ev + std::max(1, (nkr - n_ev) / 4));
            if (Th[kc] > 1.0) {
                auto pinv = [&](double th) {
                    return 0.5 * ((a + b) - (b - a) * std::cosh(std::acosh(th) / deg));
                };
                const double lam_kc = pinv(Th[kc]);
                const double lam_nev = Th[n_ev - 1] > 1.0 ? pinv(Th[n_ev - 1]) : lam_kc;
                if (lam_kc < 0.5 * a && lam_kc > two_m * two_m) {
                    a = lam_kc;
                    if (auto_deg) {
                        const double ln = (a + b - 2.0 * lam_nev) / (b - a);
                        const double ac = std::acosh(std::max(ln, 1.0 + 1e-12));
                        deg = std::max(8, std::min((int)std::ceil(4.0 / ac), 200));
                    }
                    // new filter: restart from the sum of the wanted Ritz vectors
                    std::vector<cd> yc(nkr, 0.0);
                    for (int i = 0; i < n_ev; ++i)
                        for (int r = 0; r < nkr; ++r) yc[r] += Y[(size_t)r * nkr + i];
                    HISQ_TRY(S.rotate(S.V_, nkr, yc, 1, 1, S.w_));
                    double nv = 0.0;
                    HISQ_TRY(S.norm(S.w_, &nv));
                    HISQ_TRY(vec_axpby2(S.col(S.V_, 0), 0.0, S.w_, 1.0 / nv, nullptr, 0.0, N, s));
                    theta.clear();
                    sigma.clear();
                    k0 = 0;
                    fscale = 0.0;
                    ++cut_updates;
                    continue;
                }
            }
        }
        bool conv = true;
        for (int i = 0; i < n_ev; ++i) {
            const double rho = std::abs(bl * Y[(size_t)(nkr - 1) * nkr + i]);
            if (!(rho <= tol_l * std::abs(Th[i]))) conv = false;
        }
        // thick restart, in place: keep k0n Ritz vectors (the first n_ev are the
        // wanted ones, U) and the residual direction
        const int k0n = std::min(n_ev + (nkr - n_ev) / 2, nkr - 1);
        HISQ_TRY(S.rotate_inplace(S.V_, nkr, Y, nkr, k0n));
        HISQ_HIP(hipMemcpyAsync(S.col(S.V_, k0n), S.col(S.V_, nkr), sizeof(double2) * (size_t)N,
                                hipMemcpyDeviceToDevice, s));
        HISQ_TRY(S.check_cols());
        theta.assign(Th.begin(), Th.begin() + k0n);
        sigma.resize(k0n);
        for (int i = 0; i < k0n; ++i) sigma[i] = bl * Y[(size_t)(nkr - 1) * nkr + i].real();
        k0 = k0n;
        if (!(conv || restarts == max_restarts)) continue;

        // Rayleigh-Ritz on A over U = V[0..n_ev): G = U^H A U, a block of
        // columns of A U at a time
        double2 *U = S.col(S.V_, 0, n_ev);
        HISQ_TRY(S.check_cols());
        std::vector<cd> G((size_t)n_ev * n_ev), Zg;
        {
            std::vector<cd> C;
            for (int c0 = 0; c0 < n_ev; c0 += S.tcols_) {
                const int nc = std::min(S.tcols_, n_ev - c0);
                HISQ_TRY(S.applyA(S.col(S.V_, c0, nc), S.T_, nc));
                // C[j][i] = <U_i, (A U)_{c0 + j}> = G[i][c0 + j]
                HISQ_TRY(gemm_tn(g, U, n_ev, S.T_, nc, N, nullptr, 1.0, S.coef_, s));
                C.resize((size_t)nc * n_ev);
                HISQ_HIP(hipMemcpyAsync(C.data(), S.coef_, sizeof(double2) * C.size(),
                                        hipMemcpyDeviceToHost, s));
                HISQ_HIP(hipStreamSynchronize(s));
                for (int j = 0; j < nc; ++j)
                    for (int i = 0; i < n_ev; ++i) G[(size_t)i * n_ev + c0 + j] = C[(size_t)j * n_ev + i];
            }
            // Hermitian part (rounding makes G slightly non-Hermitian)
            for (int i = 0; i < n_ev; ++i)
                for (int j = i; j < n_ev; ++j) {
                    const cd h = 0.5 * (G[(size_t)i * n_ev + j] + std::conj(G[(size_t)j * n_ev + i]));
                    G[(size_t)i * n_ev + j] = h;
                    G[(size_t)j * n_ev + i] = std::conj(h);
                }
        }
        std::vector<double> lam;
        if (small_heev(n_ev, G, lam, Zg) < 0)
            return fail(HISQ_ERR_BREAKDOWN, "eigensolve: Rayleigh-Ritz did not converge");
        // E = U Z in place, then ||A e_i - lambda_i e_i|| a block at a time
        HISQ_TRY(S.rotate_inplace(U, n_ev, Zg, n_ev, n_ev));
        double2 *E = U;
        HISQ_HIP(hipMemcpyAsync(S.dscal_, lam.data(), sizeof(double) * n_ev, hipMemcpyHostToDevice,
                                s));
        for (int c0 = 0; c0 < n_ev; c0 += S.tcols_) {
            const int nc = std::min(S.tcols_, n_ev - c0);
            HISQ_TRY(S.applyA(S.col(S.V_, c0, nc), S.T_, nc));
            HISQ_TRY(vec_col_residuals(g, S.T_, S.col(S.V_, c0, nc), S.dscal_ + c0, N, nc,
                                       S.dscal_ + n_ev + c0, s));
        }
        std::vector<double> r2(n_ev);
        HISQ_HIP(hipMemcpyAsync(r2.data(), S.dscal_ + n_ev, sizeof(double) * n_ev,
                                hipMemcpyDeviceToHost, s));
        HISQ_HIP(hipStreamSynchronize(s));
        max_res = 0.0;
        for (int i = 0; i < n_ev; ++i) max_res = std::max(max_res, std::sqrt(r2[i]));
        lam_out = lam;
        if (max_res <= tol * lam_max) {
            // Completeness: residuals cannot reveal a copy of a degenerate
            // eigenvalue that never entered the Krylov space.  Filter a random
            // vector orthogonal to the accepted ones; if its Rayleigh quotient
            // falls below the last accepted eigenvalue, it joins the basis.
            double2 *u = S.w_;
            double2 *scratch = S.col(S.T_, 0);
            HISQ_TRY(vec_random(u, N, seed + 424242 + restarts, s));
            double un = 0.0;
            for (int it = 0; it < 4; ++it) {
                if (it > 0) {
                    HISQ_TRY(S.chebyshev(u, scratch, deg, a, b));
                    HISQ_HIP(hipMemcpyAsync(u, scratch, sizeof(double2) * (size_t)N,
                                            hipMemcpyDeviceToDevice, s));
                }
                HISQ_TRY(S.orthogonalise(u, n_ev, E));
                HISQ_TRY(S.norm(u, &un));
                if (!(un > 0.0)) break;
                HISQ_TRY(vec_axpby2(u, 1.0 / un, nullptr, 0.0, nullptr, 0.0, N, s));
            }
            double lam_u = INFINITY;
            if (un > 0.0) {
                HISQ_TRY(S.applyA(u, scratch));
                cd q;
                HISQ_TRY(S.dot(u, scratch, &q));
                lam_u = q.real();
            }
            if (!(lam_u < lam[n_ev - 1] - 1e-8 * lam_max)) {
                accepted = true;
                final_status = HISQ_OK;
                break;
            }
            if (restarts == max_restarts) break;
            // restart from [accepted vectors, u]: p(A) e_i = p(lambda_i) e_i up to
            // the accepted residual, so the kept block carries no coupling
            HISQ_HIP(hipMemcpyAsync(S.col(S.V_, n_ev), u, sizeof(double2) * (size_t)N,
                                    hipMemcpyDeviceToDevice, s));
            HISQ_TRY(S.check_cols());
            theta.assign(n_ev, 0.0);
            sigma.assign(n_ev, 0.0);
            for (int i = 0; i < n_ev; ++i) theta[i] = Solver::cheb_value(lam[i], deg, a, b);
            k0 = n_ev;
            continue;
        }
        if (restarts == max_restarts) break;
        // not yet: undo the Rayleigh-Ritz rotation (U = E Z^H) so that the kept
        // block is again the Ritz basis of the restart, ask the Lanczos cycle
        // for more and continue restarting
        HISQ_TRY(S.rotate_inplace(U, n_ev, Zg, n_ev, n_ev, true));
        tol_l *= 0.1;
    }
    HISQ_TRY(S.check_cols());
    if (accepted || restarts >= max_restarts) {
        // the eigenvectors (or the best pairs found) to the caller's buffer
        if (evec_prec == HISQ_FP64)
            HISQ_HIP(hipMemcpyAsync(evecs_dev, S.V_, sizeof(double2) * (size_t)N * n_ev,
                                    hipMemcpyDeviceToDevice, s));
        else
            HISQ_TRY(convert_vectors(S.V_, HISQ_FP64, evecs_dev, HISQ_FP32, N * (int64_t)n_ev, s));
    }
    HISQ_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n_ev; ++i) evals_host[i] = lam_out[i];
    if (stats_host) {
        stats_host->restarts = restarts;
        stats_host->matvecs = S.matvecs_;
        stats_host->converged = accepted ? n_ev : 0;
        stats_host->cheb_degree = deg;
        stats_host->cheb_a = a;
        stats_host->cheb_b = b;
        stats_host->lambda_max = lam_max;
        stats_host->max_residual = max_res;
        stats_host->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (final_status != HISQ_OK)
        return fail(final_status, "eigensolve: residual target not met within max_restarts");
    return HISQ_OK;
}
