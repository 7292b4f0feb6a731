// Host-side dense Hermitian eigensolvers for the small projected matrices of
// the eigensolver: cyclic Jacobi (the Rayleigh-Ritz Gram matrix; slow for
// large n but accurate for graded matrices) and Householder + implicit QR (the
// Lanczos matrices of a thick-restart cycle, real for one vector per step,
// complex Hermitian for a block).
#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <numeric>
#include <type_traits>
#include <vector>

namespace hisq {

using cd = std::complex<double>;

// A: n x n Hermitian, row-major, overwritten.  On return w holds the
// eigenvalues in ascending order and Z (n x n, row-major) the eigenvectors as
// columns: A_in Z[:, i] = w[i] Z[:, i].  Returns the number of sweeps used, or
// -1 if the off-diagonal mass did not fall below tolerance in max_sweeps.
int heev_jacobi(int n, cd *A, double *w, cd *Z, int max_sweeps) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Z[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    auto at = [&](int i, int j) -> cd & { return A[(size_t)i * n + j]; };
    double scale = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) scale = std::max(scale, std::abs(at(i, j)));
    if (scale == 0.0) {
        for (int i = 0; i < n; ++i) w[i] = 0.0;
        return 0;
    }
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += std::norm(at(i, i));
            for (int j = i + 1; j < n; ++j) off += std::norm(at(i, j));
        }
        if (off <= 1e-34 * diag || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const cd apq = at(p, q);
                const double b = std::abs(apq);
                if (b == 0.0) continue;
                const double app = at(p, p).real(), aqq = at(q, q).real();
                // skip rotations below the resolution of both diagonal entries
                if (b < 1e-18 * (std::abs(app) + std::abs(aqq)) && sweep > 3) {
                    at(p, q) = at(q, p) = 0.0;
                    continue;
                }
                // phase: apq = b e^{i phi}; with P = diag(1, e^{-i phi}) the
                // 2x2 block becomes real [[app, b], [b, aqq]]
                const cd ph = apq / b;  // e^{i phi}
                const double tau = (aqq - app) / (2.0 * b);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // J = P R with R = [[c, s], [-s, c]]:
                //   J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
                const cd J00 = c, J01 = s;
                const cd J10 = -s * std::conj(ph), J11 = c * std::conj(ph);
                // A <- A J (columns p, q)
                for (int k = 0; k < n; ++k) {
                    const cd akp = at(k, p), akq = at(k, q);
                    at(k, p) = akp * J00 + akq * J10;
                    at(k, q) = akp * J01 + akq * J11;
                }
                // A <- J^H A (rows p, q)
                for (int k = 0; k < n; ++k) {
                    const cd apk = at(p, k), aqk = at(q, k);
                    at(p, k) = std::conj(J00) * apk + std::conj(J10) * aqk;
                    at(q, k) = std::conj(J01) * apk + std::conj(J11) * aqk;
                }
                at(p, q) = at(q, p) = 0.0;
                at(p, p) = at(p, p).real();
                at(q, q) = at(q, q).real();
                for (int k = 0; k < n; ++k) {
                    cd &zp = Z[(size_t)k * n + p], &zq = Z[(size_t)k * n + q];
                    const cd zkp = zp, zkq = zq;
                    zp = zkp * J00 + zkq * J10;
                    zq = zkp * J01 + zkq * J11;
                }
            }
        }
    }
    // sort ascending
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::vector<double> d(n);
    for (int i = 0; i < n; ++i) d[i] = at(i, i).real();
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
    std::vector<cd> Zs((size_t)n * n);
    for (int c2 = 0; c2 < n; ++c2) {
        w[c2] = d[idx[c2]];
        for (int r = 0; r < n; ++r) Zs[(size_t)r * n + c2] = Z[(size_t)r * n + idx[c2]];
    }
    std::copy(Zs.begin(), Zs.end(), Z);
    return sweep < max_sweeps ? sweep : -1;
}

// Householder tridiagonalisation followed by the implicit symmetric QR
// iteration with Wilkinson shifts (bulge chasing with Givens rotations),
// eigenvectors accumulated throughout: for the Lanczos matrices, real
// symmetric (T = double: arrowhead plus tridiagonal) or complex Hermitian
// (T = complex: arrowhead plus block tridiagonal, from the block Lanczos).
// O(n^3) with a small constant, against the O(sweeps n^3) cyclic Jacobi;
// backward stable (errors of order eps ||A||, enough for the large filtered
// Ritz values the eigensolver keeps).
// A: n x n, row-major, overwritten.  On return w holds the eigenvalues
// ascending and Z (row-major) the eigenvectors as columns.  Returns the
// number of QR steps, or -1 if an eigenvalue needed more than 60.
namespace {
inline double conj_(double x) { return x; }
inline cd conj_(cd x) { return std::conj(x); }
inline double abs_(double x) { return std::fabs(x); }
inline double abs_(cd x) { return std::abs(x); }
inline double real_(double x) { return x; }
inline double real_(cd x) { return x.real(); }

template <typename T>
int tridiag_qr(int n, T *A, double *w, T *Z) {
    constexpr bool cplx = !std::is_same<T, double>::value;
    auto a = [&](int i, int j) -> T & { return A[(size_t)i * n + j]; };
    auto z = [&](int i, int j) -> T & { return Z[(size_t)i * n + j]; };
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) z(i, j) = i == j ? 1.0 : 0.0;
    // 1. Householder: for each column k, reflect rows/columns k+1.. so that
    //    column k has a single nonzero below the diagonal.  H = I - 2 v v^H
    //    with alpha = -phase(x0) ||x|| maps x to alpha e_1.  Z accumulates the
    //    product of the reflections (Z <- Z H).
    std::vector<T> v(n), p(n), q(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;  // length of the reflected part
        double xn = 0.0;
        for (int i = 0; i < m; ++i) xn = std::hypot(xn, abs_(a(k + 1 + i, k)));
        if (xn == 0.0) continue;
        const T x0 = a(k + 1, k);
        T ph = 1.0;
        if (cplx) {
            if (abs_(x0) > 0.0) ph = x0 / abs_(x0);
        } else if (real_(x0) < 0.0) {
            ph = -1.0;
        }
        const T alpha = -xn * ph;
        for (int i = 0; i < m; ++i) v[i] = a(k + 1 + i, k);
        v[0] -= alpha;
        double vn = 0.0;
        for (int i = 0; i < m; ++i) vn = std::hypot(vn, abs_(v[i]));
        if (vn == 0.0) continue;
        for (int i = 0; i < m; ++i) v[i] /= vn;
        // on the trailing block B: B <- H B H = B - 2 v q^H - 2 q v^H with
        // p = B v, q = p - (v^H p) v (v^H p is real for Hermitian B)
        for (int i = 0; i < m; ++i) {
            T t = 0.0;
            for (int j = 0; j < m; ++j) t += a(k + 1 + i, k + 1 + j) * v[j];
            p[i] = t;
        }
        double vp = 0.0;
        for (int i = 0; i < m; ++i) vp += real_(conj_(v[i]) * p[i]);
        for (int i = 0; i < m; ++i) q[i] = p[i] - vp * v[i];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                a(k + 1 + i, k + 1 + j) -= 2.0 * (v[i] * conj_(q[j]) + q[i] * conj_(v[j]));
        a(k + 1, k) = alpha;
        a(k, k + 1) = conj_(alpha);
        for (int i = 1; i < m; ++i) a(k + 1 + i, k) = a(k, k + 1 + i) = 0.0;
        // Z <- Z H on columns k+1..
        for (int r = 0; r < n; ++r) {
            T t = 0.0;
            for (int j = 0; j < m; ++j) t += z(r, k + 1 + j) * v[j];
            t *= 2.0;
            for (int j = 0; j < m; ++j) z(r, k + 1 + j) -= t * conj_(v[j]);
        }
    }
    std::vector<double> d(n), e(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = real_(a(i, i));
    if (cplx) {
        // T = D T' D^H with D = diag(delta), delta_{k+1} = delta_k phase(e_k),
        // makes the subdiagonal of T' real (|e_k|); the eigenvectors of T are
        // D times those of T', so Z <- Z D.
        T delta = 1.0;
        for (int k = 0; k < n; ++k) {
            if (k > 0) {
                const T ek = a(k, k - 1);
                const double ae = abs_(ek);
                e[k - 1] = ae;
                if (ae > 0.0) delta *= ek / ae;
                for (int r = 0; r < n; ++r) z(r, k) *= delta;
            }
        }
    } else {
        for (int i = 0; i + 1 < n; ++i) e[i] = real_(a(i + 1, i));
    }
    // 2. Implicit QR on the unreduced blocks, from the bottom up.
    const double eps = std::numeric_limits<double>::epsilon();
    int steps = 0, m = n - 1, iters = 0;
    while (m > 0) {
        int l = m;
        while (l > 0) {
            if (std::fabs(e[l - 1]) <= eps * (std::fabs(d[l - 1]) + std::fabs(d[l]))) {
                e[l - 1] = 0.0;
                break;
            }
            --l;
        }
        if (l == m) {  // d[m] has converged
            --m;
            iters = 0;
            continue;
        }
        if (++iters > 60) return -1;
        ++steps;
        // Wilkinson shift from the trailing 2 x 2 block of [l, m]
        const double delta = 0.5 * (d[m - 1] - d[m]), bb = e[m - 1];
        const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * std::hypot(delta, bb);
        const double mu = den != 0.0 ? d[m] - bb * bb / den : d[m] - std::fabs(bb);
        double x = d[l] - mu, zz = e[l];
        for (int k = l; k < m; ++k) {
            const double r = std::hypot(x, zz);
            const double c = r != 0.0 ? x / r : 1.0, s = r != 0.0 ? zz / r : 0.0;
            if (k > l) e[k - 1] = r;
            // T <- G^T T G on rows/columns k, k+1, G = [[c, -s], [s, c]]
            const double dk = d[k], ek = e[k], dk1 = d[k + 1];
            d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
            d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
            e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
            if (k + 1 < m) {
                x = e[k];
                zz = s * e[k + 1];    // the bulge at (k+2, k)
                e[k + 1] *= c;
            }
            for (int r2 = 0; r2 < n; ++r2) {
                const T zk = z(r2, k), zk1 = z(r2, k + 1);
                z(r2, k) = c * zk + s * zk1;
                z(r2, k + 1) = -s * zk + c * zk1;
            }
        }
    }
    // 3. sort ascending
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x1, int y1) { return d[x1] < d[y1]; });
    std::vector<T> Zs((size_t)n * n);
    for (int c2 = 0; c2 < n; ++c2) {
        w[c2] = d[idx[c2]];
        for (int r = 0; r < n; ++r) Zs[(size_t)r * n + c2] = z(r, idx[c2]);
    }
    std::copy(Zs.begin(), Zs.end(), Z);
    return steps;
}
}  // namespace

int syev_qr(int n, double *A, double *w, double *Z) { return tridiag_qr<double>(n, A, w, Z); }
int heev_qr(int n, cd *A, double *w, cd *Z) { return tridiag_qr<cd>(n, A, w, Z); }

}  // namespace hisq
