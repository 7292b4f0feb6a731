// Vector kernels of the eigensolver: a counter-based random start vector,
// FP64 dot products with fixed-order reductions (partials, then a sum in block order), scaled sums, and per-column
// residual norms ||w_i - lambda_i u_i||.
#include "device_util.h"
#include "hisq_internal.h"

namespace hisq {

typedef double dvec2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int kBS = 256;

int grid_for(int64_t n) {
    int64_t nb = (n + 4 * kBS - 1) / (4 * kBS);
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    return (int)nb;
}

// splitmix64 (Steele, Lea, Flood 2014): a counter-based 64-bit mixer.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double unit_interval(uint64_t u) {
    // 53 random bits -> [-1, 1)
    return (double)(u >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(kBS) void k_random(dvec2 *__restrict__ x, int64_t n, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const uint64_t base = seed * 0x100000001b3ull + 2 * (uint64_t)i;
        x[i] = dvec2{unit_interval(splitmix64(base)), unit_interval(splitmix64(base + 1))};
    }
}

// Per-block partials of <x, y> = sum conj(x) y: real parts at [block],
// imaginary parts at [nb + block]; k_sum_rows adds them in block order.
__global__ __launch_bounds__(kBS) void k_dot(const dvec2 *__restrict__ x, const dvec2 *__restrict__ y,
                                             int64_t n, double *__restrict__ partials) {
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const dvec2 a = x[i], b = y[i];
        v[0] = fma(a.x, b.x, fma(a.y, b.y, v[0]));
        v[1] = fma(a.x, b.y, fma(-a.y, b.x, v[1]));
    }
    __shared__ double lds[2 * (kBS / kWave)];
    block_sum<2, kBS>(v, lds);
    const int nb = gridDim.x;
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = v[0];
        partials[nb + blockIdx.x] = v[1];
    }
}

// out[q] = sum of row q of partials ([rows][nb]) in block order; one wave per row.
__global__ __launch_bounds__(kBS) void k_sum_rows(const double *__restrict__ partials, int nb,
                                                  int rows, double *__restrict__ out) {
    const int q = blockIdx.x * (kBS / kWave) + threadIdx.x / kWave;
    if (q >= rows) return;
    const int lane = threadIdx.x & (kWave - 1);
    double v = 0.0;
    for (int i = lane; i < nb; i += kWave) v += partials[(int64_t)q * nb + i];
    v = wave_sum(v);
    if (lane == 0) out[q] = v;
}

// y = a y + b1 x1 + b2 x2 (x1, x2 optional)
__global__ __launch_bounds__(kBS) void k_axpby2(dvec2 *__restrict__ y, double a,
                                                const dvec2 *__restrict__ x1, double b1,
                                                const dvec2 *__restrict__ x2, double b2,
                                                int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        dvec2 v = y[i] * a;
        if (x1) {
            const dvec2 u = x1[i];
            v.x = fma(b1, u.x, v.x);
            v.y = fma(b1, u.y, v.y);
        }
        if (x2) {
            const dvec2 u = x2[i];
            v.x = fma(b2, u.x, v.x);
            v.y = fma(b2, u.y, v.y);
        }
        y[i] = v;
    }
}

// Per-block partials of ||W_i - lam_i U_i||^2 over k columns of n complex
// (grid.y = column), stored as [k][gridDim.x].
__global__ __launch_bounds__(kBS) void k_colres(const dvec2 *__restrict__ W, const dvec2 *__restrict__ U,
                                                const double *__restrict__ lam, int64_t n,
                                                double *__restrict__ partials) {
    const int col = blockIdx.y;
    const double l = lam[col];
    double v[1] = {0.0};
    const int64_t off = col * n;
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const dvec2 w = W[off + i], u = U[off + i];
        const double rx = fma(-l, u.x, w.x), ry = fma(-l, u.y, w.y);
        v[0] = fma(rx, rx, fma(ry, ry, v[0]));
    }
    __shared__ double lds[kBS / kWave];
    block_sum<1, kBS>(v, lds);
    if (threadIdx.x == 0) partials[(int64_t)col * gridDim.x + blockIdx.x] = v[0];
}

double *reduce_buffer(hisq_gauge_s *g, size_t nvals, hisq_status *st) {
    void *p = nullptr;
    *st = g->ws.get("vec_partials", sizeof(double) * nvals, &p);
    return static_cast<double *>(p);
}

hisq_status sum_rows(const double *partials, int nb, int rows, double *out, hipStream_t s) {
    const int per = kBS / kWave;
    hipLaunchKernelGGL(k_sum_rows, dim3((rows + per - 1) / per), dim3(kBS), 0, s, partials, nb,
                       rows, out);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

}  // namespace

hisq_status vec_random(double2 *x, int64_t n, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_random, dim3(grid_for(n)), dim3(kBS), 0, s, reinterpret_cast<dvec2 *>(x),
                       n, seed);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status vec_dot(hisq_gauge_s *g, const double2 *x, const double2 *y, int64_t n, double *out,
                    hipStream_t s) {
    const int nb = grid_for(n);
    hisq_status st = HISQ_OK;
    double *partials = reduce_buffer(g, 2 * (size_t)nb, &st);
    HISQ_TRY(st);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kBS), 0, s, reinterpret_cast<const dvec2 *>(x),
                       reinterpret_cast<const dvec2 *>(y), n, partials);
    HISQ_HIP(hipGetLastError());
    return sum_rows(partials, nb, 2, out, s);
}

hisq_status vec_axpby2(double2 *y, double a, const double2 *x1, double b1, const double2 *x2,
                       double b2, int64_t n, hipStream_t s) {
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_axpby2, dim3(grid_for(n)), dim3(kBS), 0, s, reinterpret_cast<dvec2 *>(y), a,
                       reinterpret_cast<const dvec2 *>(x1), b1,
                       reinterpret_cast<const dvec2 *>(x2), b2, n);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status vec_col_residuals(hisq_gauge_s *g, const double2 *W, const double2 *U,
                              const double *lam_dev, int64_t n, int k, double *out_dev,
                              hipStream_t s) {
    const int nb = std::max(1, grid_for(n) / 4);
    hisq_status st = HISQ_OK;
    double *partials = reduce_buffer(g, (size_t)nb * k, &st);
    HISQ_TRY(st);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_colres, dim3(nb, k), dim3(kBS), 0, s, reinterpret_cast<const dvec2 *>(W),
                       reinterpret_cast<const dvec2 *>(U), lam_dev, n, partials);
    HISQ_HIP(hipGetLastError());
    return sum_rows(partials, nb, k, out_dev, s);
}

}  // namespace hisq
