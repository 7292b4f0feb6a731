// Host-side dense Hermitian eigensolver (cyclic Jacobi) for the small
// projected matrices of the eigensolver: the Lanczos arrowhead/tridiagonal
// matrix of a thick-restart cycle and the Rayleigh-Ritz Gram matrix.
// Jacobi is slow for large n but accurate for graded matrices, which the
// Chebyshev-filtered Lanczos matrices are.
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
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

}  // namespace hisq
