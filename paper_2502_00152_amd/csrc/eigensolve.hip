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
//   3. Thick-restart Lanczos on p(A), one vector or a block of nb vectors per
//      step (block Lanczos: the filter is applied to nb vectors in one
//      multi-RHS stencil launch per half stencil, which reads the links once
//      for all of them), classical Gram-Schmidt applied twice against the
//      whole basis, a block orthonormalised by Cholesky QR applied twice.
//      After each cycle the small projected matrix (arrowhead of the kept
//      Ritz values and their couplings, then tridiagonal, or block
//      tridiagonal for nb > 1) is diagonalised on the host, the Ritz vectors
//      of the kept part become the new leading basis and the residual vector
//      (block) the next one.
//   4. When the n_ev wanted Ritz values have residuals below tol (relative to
//      each Ritz value), form the Ritz vectors, apply A to them, diagonalise
//      the Gram matrix U^H A U on the host, rotate, and accept when every
//      ||A v - lambda v|| <= tol * lambda_max; otherwise tighten and go on.
//
// Memory: one FP64 basis of n_kr + nb vectors.  Basis rotations V <- V Y are
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
int heev_qr(int n, std::complex<double> *A, double *w, std::complex<double> *Z);
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
                                             "eig_t", "eig_coef", "eig_scal"};

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
    double2 *w_ = nullptr, *y1_ = nullptr, *y2_ = nullptr, *t_ = nullptr;  // nb_ columns each
    double2 *coef_ = nullptr;  // device complex coefficients (GEMM operands)
    double *dscal_ = nullptr;  // device scalars
    double *hscal_ = nullptr;  // pinned host mirror
    Pinned pin_;
    int matvecs_ = 0;
    int gs_passes_ = 0;  // Gram-Schmidt passes (for the statistics)
    int nkr_ = 0;
    int nb_ = 1;           // Lanczos block size
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

    hisq_status alloc(int nkr, int n_ev, int nb) {
        nkr_ = nkr;
        nb_ = nb;
        void *p = nullptr;
        const size_t vb = sizeof(double2) * (size_t)N_;
        cols_ = nkr + nb;
        tcols_ = std::max(std::min(n_ev, 32), nb);
        // rows of one block of an in-place rotation of up to nkr columns
        rows_blk_ = std::max<int64_t>(8, (int64_t)tcols_ * N_ / nkr / 8 * 8);
        rows_blk_ = std::min<int64_t>(rows_blk_, N_);
        HISQ_TRY(g_->ws.get("eig_V", vb * cols_, &p));
        V_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_T", std::max(vb * tcols_, sizeof(double2) * (size_t)rows_blk_ * nkr),
                            &p));
        T_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_w", vb * nb, &p));
        w_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_y1", vb * nb, &p));
        y1_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_y2", vb * nb, &p));
        y2_ = static_cast<double2 *>(p);
        HISQ_TRY(g_->ws.get("eig_t", vb * nb, &p));
        t_ = static_cast<double2 *>(p);
        coef_cap_ = (size_t)(nkr + nb) * std::max(nkr + nb, n_ev) + 64;
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

    // w = T_d(l(A)) v with l(x) = (a + b - 2x) / (b - a), for nrhs <= nb_
    // consecutive vectors (one multi-RHS half-stencil launch per half)
    hisq_status chebyshev(const double2 *v, double2 *w, int d, double a, double b, int nrhs = 1) {
        if (nrhs < 1 || nrhs > nb_) return fail(HISQ_ERR_INVALID_ARG, "eigensolve: filter block");
        const double s1 = (a + b) / (b - a), s2 = -2.0 / (b - a);
        const double m2 = two_m_ * two_m_;
        double2 *t = t_;
        // y1 = l(A) v = (s1 + s2 m2) v - s2 D_eo D_oe v
        double2 *prev = nullptr, *cur = nullptr;
        {
            double2 *dst = d == 1 ? w : y1_;
            HISQ_TRY(launch_dslash(g_, 1, v, t, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE,
                                   nullptr, nullptr, s_));
            HISQ_TRY(launch_dslash(g_, 0, t, dst, nrhs, v, s1 + s2 * m2, nullptr, 0.0, -s2,
                                   FIN_NONE, nullptr, nullptr, s_));
            matvecs_ += nrhs;
            prev = const_cast<double2 *>(v);
            cur = dst;
        }
        // y_{i+1} = 2 l(A) y_i - y_{i-1}
        for (int i = 1; i < d; ++i) {
            double2 *dst = (i == d - 1) ? w : (prev == v ? y2_ : prev);
            HISQ_TRY(launch_dslash(g_, 1, cur, t, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE,
                                   nullptr, nullptr, s_));
            HISQ_TRY(launch_dslash(g_, 0, t, dst, nrhs, cur, 2.0 * (s1 + s2 * m2), prev, -1.0,
                                   -2.0 * s2, FIN_NONE, nullptr, nullptr, s_));
            matvecs_ += nrhs;
            prev = cur;
            cur = dst;
        }
        return HISQ_OK;
    }

    // host <- device coefficients (n complex), synchronising the stream
    hisq_status coef_to_host(std::vector<cd> &C, size_t n) {
        if (n > coef_cap_) return fail(HISQ_ERR_INVALID_ARG, "eigensolve: coefficient buffer");
        C.resize(n);
        HISQ_HIP(hipMemcpyAsync(C.data(), coef_, sizeof(double2) * n, hipMemcpyDeviceToHost, s_));
        HISQ_HIP(hipStreamSynchronize(s_));
        return HISQ_OK;
    }
    hisq_status coef_to_device(const std::vector<cd> &C) {
        if (C.size() > coef_cap_) return fail(HISQ_ERR_INVALID_ARG, "eigensolve: coefficient buffer");
        HISQ_HIP(hipMemcpyAsync(coef_, C.data(), sizeof(double2) * C.size(), hipMemcpyHostToDevice,
                                s_));
        HISQ_HIP(hipStreamSynchronize(s_));  // C is pageable and may go out of scope
        return HISQ_OK;
    }

    // W (n columns) -= Q[0..j) (Q[0..j)^H W), twice: classical Gram-Schmidt
    // of a block, each pass one pair of tall-skinny products
    hisq_status project_out(double2 *W, int n, int j, const double2 *Q) {
        if (j <= 0) return HISQ_OK;
        for (int pass = 0; pass < 2; ++pass) {
            HISQ_TRY(gemm_tn(g_, Q, j, W, n, N_, nullptr, -1.0, coef_, s_));
            HISQ_TRY(gemm_nn(Q, j, coef_, n, N_, 1.0, W, s_));
            ++gs_passes_;
        }
        return HISQ_OK;
    }

    // Gram matrix G = W^H W of n columns on the host (row-major, G[i][c] = <W_i, W_c>)
    hisq_status gram(const double2 *W, int n, std::vector<cd> &G) {
        HISQ_TRY(gemm_tn(g_, W, n, W, n, N_, nullptr, 1.0, coef_, s_));
        std::vector<cd> C;
        HISQ_TRY(coef_to_host(C, (size_t)n * n));
        G.assign((size_t)n * n, 0.0);
        for (int c = 0; c < n; ++c)
            for (int i = 0; i < n; ++i) G[(size_t)i * n + c] = C[(size_t)c * n + i];
        return HISQ_OK;
    }

    // Cholesky G = R^H R (R upper triangular, row-major).  False when a pivot
    // falls below rel * (largest diagonal entry of G) or below floor: the
    // columns are too close to dependent for Cholesky QR to orthonormalise
    // them to working precision.
    static bool cholesky(int n, const std::vector<cd> &G, std::vector<cd> &R, double rel,
                         double floor) {
        R.assign((size_t)n * n, 0.0);
        double gmax = 0.0;
        for (int i = 0; i < n; ++i) gmax = std::max(gmax, G[(size_t)i * n + i].real());
        for (int i = 0; i < n; ++i) {
            double d = G[(size_t)i * n + i].real();
            for (int k = 0; k < i; ++k) d -= std::norm(R[(size_t)k * n + i]);
            if (!(d > rel * gmax) || !(d > floor)) return false;
            const double rii = std::sqrt(d);
            R[(size_t)i * n + i] = rii;
            for (int c = i + 1; c < n; ++c) {
                cd v = G[(size_t)i * n + c];
                for (int k = 0; k < i; ++k) v -= std::conj(R[(size_t)k * n + i]) * R[(size_t)k * n + c];
                R[(size_t)i * n + c] = v / rii;
            }
        }
        return true;
    }

    // Orthonormalise the n columns of W (already orthogonal to V[0..j)) into
    // V[j..j+n): W = V[j..j+n) R with R upper triangular (host, row-major).
    // Cholesky QR twice (R = R2 R1); when the columns are nearly dependent,
    // column by column Gram-Schmidt against V[0..j+c) instead, a column that
    // vanishes (below 1e-12 scale) replaced by a random vector orthogonal to
    // the basis, with a zero diagonal entry in R.  W is clobbered.
    hisq_status block_qr(double2 *W, int n, int j, std::vector<cd> &R, double scale,
                         uint64_t seed) {
        double2 *Q = col(V_, j, n);
        HISQ_TRY(check_cols());
        std::vector<cd> G, R1, R2, C;
        HISQ_TRY(gram(W, n, G));
        const double floor = (1e-12 * scale) * (1e-12 * scale);
        if (cholesky(n, G, R1, 1e-12, floor)) {
            // Q = W R1^{-1}, then W = Q R2^{-1} back into Q
            auto inv_upper = [n](const std::vector<cd> &Rm) {
                std::vector<cd> X((size_t)n * n, 0.0);
                for (int c = 0; c < n; ++c) {
                    X[(size_t)c * n + c] = 1.0 / Rm[(size_t)c * n + c];
                    for (int i = c - 1; i >= 0; --i) {
                        cd v = 0.0;
                        for (int k = i + 1; k <= c; ++k) v += Rm[(size_t)i * n + k] * X[(size_t)k * n + c];
                        X[(size_t)i * n + c] = -v / Rm[(size_t)i * n + i];
                    }
                }
                return X;
            };
            auto apply = [&](const double2 *src, const std::vector<cd> &X, double2 *dst) {
                // dst_c = sum_i src_i X[i][c]: gemm coefficient C[c][i] = X[i][c]
                C.assign((size_t)n * n, 0.0);
                for (int c = 0; c < n; ++c)
                    for (int i = 0; i < n; ++i) C[(size_t)c * n + i] = X[(size_t)i * n + c];
                HISQ_TRY(coef_to_device(C));
                return gemm_nn(src, n, coef_, n, N_, 0.0, dst, s_);
            };
            HISQ_TRY(apply(W, inv_upper(R1), Q));
            HISQ_TRY(gram(Q, n, G));
            if (cholesky(n, G, R2, 1e-6, 0.0)) {
                HISQ_TRY(apply(Q, inv_upper(R2), W));
                HISQ_HIP(hipMemcpyAsync(Q, W, sizeof(double2) * (size_t)N_ * n,
                                        hipMemcpyDeviceToDevice, s_));
                R.assign((size_t)n * n, 0.0);
                for (int i = 0; i < n; ++i)
                    for (int c = i; c < n; ++c) {
                        cd v = 0.0;
                        for (int k = i; k <= c; ++k) v += R2[(size_t)i * n + k] * R1[(size_t)k * n + c];
                        R[(size_t)i * n + c] = v;
                    }
                return HISQ_OK;
            }
            // W is untouched: fall back to Gram-Schmidt from it
        }
        R.assign((size_t)n * n, 0.0);
        for (int c = 0; c < n; ++c) {
            double2 *wc = W + (size_t)c * N_;
            for (int pass = 0; pass < 2 && j + c > 0; ++pass) {
                HISQ_TRY(gemm_tn(g_, V_, j + c, wc, 1, N_, nullptr, -1.0, coef_, s_));
                HISQ_TRY(coef_to_host(C, (size_t)(j + c)));
                for (int i = 0; i < c; ++i) R[(size_t)i * n + c] -= C[(size_t)j + i];
                HISQ_TRY(gemm_nn(V_, j + c, coef_, 1, N_, 1.0, wc, s_));
                ++gs_passes_;
            }
            double nrm = 0.0;
            HISQ_TRY(norm(wc, &nrm));
            if (!std::isfinite(nrm)) return fail(HISQ_ERR_NAN, "eigensolve: NaN in the Lanczos block");
            if (nrm <= 1e-12 * scale) {
                HISQ_TRY(vec_random(wc, N_, seed + 31 * (uint64_t)c, s_));
                HISQ_TRY(orthogonalise(wc, j + c));
                HISQ_TRY(norm(wc, &nrm));
                if (!(nrm > 0.0)) return fail(HISQ_ERR_BREAKDOWN, "eigensolve: basis exhausted");
                R[(size_t)c * n + c] = 0.0;
            } else {
                R[(size_t)c * n + c] = nrm;
            }
            HISQ_TRY(vec_axpby2(Q + (size_t)c * N_, 0.0, wc, 1.0 / nrm, nullptr, 0.0, N_, s_));
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
// real symmetric matrices (the Lanczos matrices of one vector per step) go to
// the Householder + implicit QR solver (O(n^3), 0.6 s at n = 512 against 11 s
// for Jacobi), complex ones to the complex Householder + QR solver when `qr`
// is set (the block Lanczos matrices), else to cyclic Jacobi (the
// Rayleigh-Ritz Gram matrix).
int small_heev(int n, std::vector<cd> &A, std::vector<double> &w, std::vector<cd> &Z,
               bool qr = false) {
    w.assign(n, 0.0);
    Z.assign((size_t)n * n, 0.0);
    bool real = true;
    for (const cd &v : A) real = real && v.imag() == 0.0;
    if (!real) return qr ? heev_qr(n, A.data(), w.data(), Z.data())
                         : heev_jacobi(n, A.data(), w.data(), Z.data(), 100);
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
    for (int k = 0; k < 7; ++k)
        if (params->reserved[k]) return fail(HISQ_ERR_INVALID_ARG, "reserved fields must be 0");
    const int64_t N = 3 * (int64_t)g->geom.vh;
    if (n_ev < 1 || n_ev >= N) return fail(HISQ_ERR_INVALID_ARG, "n_ev must be in [1, 3*Vh)");
    if (params->block < 0 || params->block > 32)
        return fail(HISQ_ERR_INVALID_ARG, "block must be in [0, 32]");
    const int nb = std::max(1, params->block);
    int nkr = params->n_kr;
    if (nkr <= 0) {
        nkr = std::max(std::max(2 * n_ev, n_ev + 32), n_ev + 2 * nb);
        nkr = (nkr + nb - 1) / nb * nb;
        nkr = (int)std::min<int64_t>(nkr, N - nb);
    }
    // every cycle must end with at least n_ev + nb vectors (n_ev < n_kr for
    // one vector per step), and the basis holds n_kr + nb
    if (nkr < n_ev + 2 * nb - 1 || nkr + nb > N)
        return fail(HISQ_ERR_INVALID_ARG,
                    nb == 1 ? "need n_ev < n_kr < 3*Vh"
                            : "need n_ev + 2 block - 1 <= n_kr <= 3*Vh - block");
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
    HISQ_TRY(S.alloc(nkr, n_ev, nb));
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
        // start the filtered iteration from sums of the lowest pilot Ritz
        // vectors: column c of the start block sums those with i = c mod nb
        Vstart_coef.assign((size_t)m * nb, 0.0);
        for (int i = 0; i < n_ev; ++i)
            for (int r = 0; r < m; ++r) Vstart_coef[(size_t)r * nb + i % nb] += Z[(size_t)r * m + i];
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
    std::vector<cd> R, Bprev, Cc;  // R factors of block QRs; host coefficients
    HISQ_TRY(S.rotate(S.V_, m, Vstart_coef, nb, nb, S.w_));
    for (int c = n_ev; c < nb; ++c)
        HISQ_TRY(vec_random(S.w_ + (size_t)c * N, N, seed + 2000 + c, s));
    HISQ_TRY(S.block_qr(S.w_, nb, 0, R, 0.0, seed + 3000));
    std::vector<double> theta;  // kept Ritz values of p(A), k0 of them
    std::vector<cd> sigma;      // their couplings to the next block: nb x k0, row-major
    int k0 = 0, restarts = 0;
    double tol_l = tol, max_res = INFINITY;
    bool accepted = false;
    std::vector<double> lam_out(n_ev, 0.0);
    hisq_status final_status = HISQ_ERR_NOT_CONVERGED;
    double fscale = 0.0;
    int cut_updates = 0;
    for (; restarts <= max_restarts; ++restarts) {
        // this cycle extends the basis by whole blocks to mc <= n_kr vectors
        const int mc = k0 + nb * ((nkr - k0) / nb);
        // projected matrix T = V^H p(A) V: arrowhead (kept Ritz values and
        // their couplings) + block tridiagonal (diagonal blocks V_j^H p(A) V_j,
        // off-diagonal blocks the R factors of the block QRs)
        std::vector<cd> T((size_t)mc * mc, 0.0), Z;
        for (int i = 0; i < k0; ++i) {
            T[(size_t)i * mc + i] = theta[i];
            for (int c = 0; c < nb; ++c) {
                T[(size_t)(k0 + c) * mc + i] = sigma[(size_t)c * k0 + i];
                T[(size_t)i * mc + k0 + c] = std::conj(sigma[(size_t)c * k0 + i]);
            }
        }
        for (int j = k0; j < mc; j += nb) {
            double2 *Vj = S.col(S.V_, j, nb);
            HISQ_TRY(S.check_cols());
            HISQ_TRY(S.chebyshev(Vj, S.w_, deg, a, b, nb));
            if (j == k0 && k0 > 0) {
                // W -= V[0..k0) T[0..k0)[k0..k0+nb): the arrowhead couplings
                Cc.assign((size_t)nb * k0, 0.0);
                for (int c = 0; c < nb; ++c)
                    for (int i = 0; i < k0; ++i)
                        Cc[(size_t)c * k0 + i] = -std::conj(sigma[(size_t)c * k0 + i]);
                HISQ_TRY(S.coef_to_device(Cc));
                HISQ_TRY(gemm_nn(S.V_, k0, S.coef_, nb, N, 1.0, S.w_, s));
            } else if (j > k0) {
                // W -= V[j-nb..j) B^H, B the R factor that made V[j..j+nb)
                Cc.assign((size_t)nb * nb, 0.0);
                for (int c = 0; c < nb; ++c)
                    for (int r = 0; r < nb; ++r)
                        Cc[(size_t)c * nb + r] = -std::conj(Bprev[(size_t)c * nb + r]);
                HISQ_TRY(S.coef_to_device(Cc));
                HISQ_TRY(gemm_nn(S.col(S.V_, j - nb, nb), nb, S.coef_, nb, N, 1.0, S.w_, s));
            }
            // diagonal block: Hermitian part of V_j^H W, then W -= V_j (that block)
            HISQ_TRY(gemm_tn(g, Vj, nb, S.w_, nb, N, nullptr, 1.0, S.coef_, s));
            HISQ_TRY(S.coef_to_host(Cc, (size_t)nb * nb));  // Cc[c][i] = <V_{j+i}, W_c>
            std::vector<cd> Ad((size_t)nb * nb);
            for (int i = 0; i < nb; ++i)
                for (int c = 0; c < nb; ++c)
                    Ad[(size_t)i * nb + c] =
                        0.5 * (Cc[(size_t)c * nb + i] + std::conj(Cc[(size_t)i * nb + c]));
            for (int i = 0; i < nb; ++i) {
                fscale = std::max(fscale, std::abs(Ad[(size_t)i * nb + i].real()));
                for (int c = 0; c < nb; ++c) T[(size_t)(j + i) * mc + j + c] = Ad[(size_t)i * nb + c];
            }
            for (int c = 0; c < nb; ++c)
                for (int i = 0; i < nb; ++i) Cc[(size_t)c * nb + i] = -Ad[(size_t)i * nb + c];
            HISQ_TRY(S.coef_to_device(Cc));
            HISQ_TRY(gemm_nn(Vj, nb, S.coef_, nb, N, 1.0, S.w_, s));
            // full re-orthogonalisation, then the next block: W = V[j+nb..j+2nb) R
            HISQ_TRY(S.project_out(S.w_, nb, j + nb, S.V_));
            HISQ_TRY(S.block_qr(S.w_, nb, j + nb, R, fscale, seed + 7777 + 131 * restarts + j));
            if (j + nb < mc)
                for (int c = 0; c < nb; ++c)
                    for (int r = 0; r < nb; ++r) {
                        T[(size_t)(j + nb + c) * mc + j + r] = R[(size_t)c * nb + r];
                        T[(size_t)(j + r) * mc + j + nb + c] = std::conj(R[(size_t)c * nb + r]);
                    }
            Bprev = R;
            report(restarts, j);
        }
        HISQ_TRY(S.check_cols());
        std::vector<double> th;
        if (small_heev(mc, T, th, Z, true) < 0)
            return fail(HISQ_ERR_BREAKDOWN, "eigensolve: projected eigenproblem did not converge");
        // descending order: the largest filtered values belong to the smallest of A
        std::vector<double> Th(mc);
        std::vector<cd> Y((size_t)mc * mc);
        for (int c2 = 0; c2 < mc; ++c2) {
            Th[c2] = th[mc - 1 - c2];
            for (int r = 0; r < mc; ++r) Y[(size_t)r * mc + c2] = Z[(size_t)r * mc + (mc - 1 - c2)];
        }
        // coupling of Ritz vector i to residual direction c: (B Y_last)[c][i],
        // Y_last the last nb rows of Y, B the R factor of the last block QR
        auto coupling = [&](int c, int i) {
            cd v = 0.0;
            for (int r = 0; r < nb; ++r) v += Bprev[(size_t)c * nb + r] * Y[(size_t)(mc - nb + r) * mc + i];
            return v;
        };
        // Tighten the cut.  If the (kc+1)-th largest Ritz value of p(A) exceeds 1,
        // interlacing puts at least kc+1 eigenvalues of A at or below
        // p^{-1}(that value), so it is a valid cut with n_ev < kc + 1.
        if (auto_a && cut_updates < 4 && restarts < max_restarts) {
            const int kc = std::min(mc - 1, n_ev + std::max(1, (mc - n_ev) / 4));
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
                    // new filter: restart from sums of the wanted Ritz vectors
                    std::vector<cd> yc((size_t)mc * nb, 0.0);
                    for (int i = 0; i < n_ev; ++i)
                        for (int r = 0; r < mc; ++r) yc[(size_t)r * nb + i % nb] += Y[(size_t)r * mc + i];
                    HISQ_TRY(S.rotate(S.V_, mc, yc, nb, nb, S.w_));
                    for (int c = n_ev; c < nb; ++c)
                        HISQ_TRY(vec_random(S.w_ + (size_t)c * N, N, seed + 5000 + 17 * cut_updates + c, s));
                    HISQ_TRY(S.block_qr(S.w_, nb, 0, R, 0.0, seed + 6000 + cut_updates));
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
            double rho2 = 0.0;
            for (int c = 0; c < nb; ++c) rho2 += std::norm(coupling(c, i));
            if (!(std::sqrt(rho2) <= tol_l * std::abs(Th[i]))) conv = false;
        }
        // thick restart, in place: keep k0n Ritz vectors (the first n_ev are the
        // wanted ones, U) and the residual block
        const int k0n = std::min(n_ev + (mc - n_ev) / 2, mc - nb);
        HISQ_TRY(S.rotate_inplace(S.V_, mc, Y, mc, k0n));
        HISQ_HIP(hipMemcpyAsync(S.col(S.V_, k0n, nb), S.col(S.V_, mc, nb),
                                sizeof(double2) * (size_t)N * nb, hipMemcpyDeviceToDevice, s));
        HISQ_TRY(S.check_cols());
        theta.assign(Th.begin(), Th.begin() + k0n);
        sigma.assign((size_t)nb * k0n, 0.0);
        for (int c = 0; c < nb; ++c)
            for (int i = 0; i < k0n; ++i) sigma[(size_t)c * k0n + i] = coupling(c, i);
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
            // block orthogonal to the accepted vectors (in the basis columns
            // after them); if the smallest Rayleigh-Ritz value of A on it falls
            // below the last accepted eigenvalue, it joins the basis.
            double2 *Vu = S.col(S.V_, n_ev, nb);
            HISQ_TRY(S.check_cols());
            HISQ_TRY(vec_random(S.w_, N * nb, seed + 424242 + restarts, s));
            for (int it = 0; it < 4; ++it) {
                if (it > 0) HISQ_TRY(S.chebyshev(Vu, S.w_, deg, a, b, nb));
                HISQ_TRY(S.project_out(S.w_, nb, n_ev, E));
                HISQ_TRY(S.block_qr(S.w_, nb, n_ev, R, 0.0, seed + 525252 + 7 * restarts + it));
            }
            double lam_u = INFINITY;
            {
                HISQ_TRY(S.applyA(Vu, S.T_, nb));
                HISQ_TRY(gemm_tn(g, Vu, nb, S.T_, nb, N, nullptr, 1.0, S.coef_, s));
                HISQ_TRY(S.coef_to_host(Cc, (size_t)nb * nb));
                std::vector<cd> Gu((size_t)nb * nb), Zu;
                for (int i = 0; i < nb; ++i)
                    for (int c = 0; c < nb; ++c)
                        Gu[(size_t)i * nb + c] =
                            0.5 * (Cc[(size_t)c * nb + i] + std::conj(Cc[(size_t)i * nb + c]));
                std::vector<double> wu;
                if (small_heev(nb, Gu, wu, Zu, true) < 0)
                    return fail(HISQ_ERR_BREAKDOWN, "eigensolve: completeness check did not converge");
                lam_u = wu[0];
            }
            if (!(lam_u < lam[n_ev - 1] - 1e-8 * lam_max)) {
                accepted = true;
                final_status = HISQ_OK;
                break;
            }
            if (restarts == max_restarts) break;
            // restart from [accepted vectors, the block]: p(A) e_i = p(lambda_i)
            // e_i up to the accepted residual, so the kept part carries no coupling
            theta.assign(n_ev, 0.0);
            sigma.assign((size_t)nb * n_ev, 0.0);
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
