// Vector kernels of the eigensolver: a counter-based random start vector,
// FP64 dot products with fixed-order reductions, scaled sums, and per-column
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

// out[0] + i out[1] = <x, y> = sum conj(x) y
__global__ __launch_bounds__(kBS) void k_dot(const dvec2 *__restrict__ x, const dvec2 *__restrict__ y,
                                             int64_t n, double *out, Reduce red) {
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
        red.partials[blockIdx.x] = v[0];
        red.partials[nb + blockIdx.x] = v[1];
    }
    if (last_block_arrive(red.counter, nb)) {
        __shared__ double w[kBS / kWave];
        const double re = sum_partials<kBS>(red.partials, nb, w);
        const double im = sum_partials<kBS>(red.partials + nb, nb, w);
        if (threadIdx.x == 0) {
            out[0] = re;
            out[1] = im;
        }
        last_block_done(red.counter);
    }
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

// out[i] = ||W_i - lam_i U_i||^2 over k columns of n complex (grid.y = column)
__global__ __launch_bounds__(kBS) void k_colres(const dvec2 *__restrict__ W, const dvec2 *__restrict__ U,
                                                const double *__restrict__ lam, int64_t n, int k,
                                                double *out, Reduce red) {
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
    const int nb = gridDim.x;
    if (threadIdx.x == 0) red.partials[(int64_t)col * nb + blockIdx.x] = v[0];
    if (last_block_arrive(red.counter, gridDim.x * gridDim.y)) {
        __shared__ double w2[kBS / kWave];
        for (int c = 0; c < k; ++c) {
            const double s = sum_partials<kBS>(red.partials + (int64_t)c * nb, nb, w2);
            if (threadIdx.x == 0) out[c] = s;
        }
        last_block_done(red.counter);
    }
}

hisq_status reduce_buffers(hisq_gauge_s *g, size_t nvals, Reduce &red) {
    void *p = nullptr;
    HISQ_TRY(g->ws.get("vec_partials", sizeof(double) * nvals, &p));
    red.partials = static_cast<double *>(p);
    HISQ_TRY(g->ws.get("vec_counter", 256, &p));
    red.counter = static_cast<unsigned *>(p);
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
    Reduce red{};
    const int nb = grid_for(n);
    HISQ_TRY(reduce_buffers(g, 2 * (size_t)nb, red));
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kBS), 0, s, reinterpret_cast<const dvec2 *>(x),
                       reinterpret_cast<const dvec2 *>(y), n, out, red);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
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
    Reduce red{};
    const int nb = std::max(1, grid_for(n) / 4);
    HISQ_TRY(reduce_buffers(g, (size_t)nb * k, red));
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_colres, dim3(nb, k), dim3(kBS), 0, s, reinterpret_cast<const dvec2 *>(W),
                       reinterpret_cast<const dvec2 *>(U), lam_dev, n, k, out_dev, red);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

}  // namespace hisq
