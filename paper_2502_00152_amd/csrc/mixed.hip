// Kernels of the mixed-precision CG: precision conversion, the reliable
// update (x += x_sloppy, r = b - A x in FP64) and the search-direction
// restart after it, each applied to the right-hand sides selected by a
// per-RHS mask.
#include "device_util.h"
#include "hisq_internal.h"

namespace hisq {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int kBS = 256;

int grid_x(int64_t n) {
    int64_t nb = (n + 4 * kBS - 1) / (4 * kBS);
    return (int)std::max<int64_t>(1, std::min<int64_t>(nb, 1024));
}

#define GRID_STRIDE(i) \
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS)

// dst = (float) src, for masked RHS
__global__ __launch_bounds__(kBS) void k_to_f32(const dvec2 *__restrict__ src, fvec2 *__restrict__ dst,
                                                int64_t n, const int *__restrict__ mask) {
    const int rhs = blockIdx.y;
    if (mask && !mask[rhs]) return;
    const int64_t off = rhs * n;
    GRID_STRIDE(i) {
        const dvec2 v = src[off + i];
        dst[off + i] = fvec2{(float)v.x, (float)v.y};
    }
}

// x += (double) xs; xs = 0, for masked RHS
__global__ __launch_bounds__(kBS) void k_accum_x(dvec2 *__restrict__ x, fvec2 *__restrict__ xs,
                                                 int64_t n, const int *__restrict__ mask) {
    const int rhs = blockIdx.y;
    if (mask && !mask[rhs]) return;
    const int64_t off = rhs * n;
    GRID_STRIDE(i) {
        const fvec2 a = xs[off + i];
        dvec2 v = x[off + i];
        v.x += (double)a.x;
        v.y += (double)a.y;
        x[off + i] = v;
        xs[off + i] = fvec2{0.0f, 0.0f};
    }
}

// r = b - Ax and per-block partials of ||r||^2 for masked RHS (0 for the
// others); k_resid_sum adds each RHS's partials in block order.  (No
// cross-block synchronisation: a device-scope fence per block writes back L2
// on this multi-XCD chip and costs more than the pass itself.)
__global__ __launch_bounds__(kBS) void k_resid(const dvec2 *__restrict__ b, const dvec2 *__restrict__ Ax,
                                               dvec2 *__restrict__ r, int64_t n,
                                               const int *__restrict__ mask, double *partials) {
    const int rhs = blockIdx.y;
    const int64_t off = rhs * n;
    double v[1] = {0.0};
    if (!mask || mask[rhs]) {
        GRID_STRIDE(i) {
            const dvec2 rr = b[off + i] - Ax[off + i];
            r[off + i] = rr;
            v[0] = fma(rr.x, rr.x, fma(rr.y, rr.y, v[0]));
        }
    }
    __shared__ double lds[kBS / kWave];
    block_sum<1, kBS>(v, lds);
    if (threadIdx.x == 0) partials[(int64_t)rhs * gridDim.x + blockIdx.x] = v[0];
}

// out[q] = sum of the nb partials of RHS q in block order; one wave per RHS.
__global__ __launch_bounds__(kBS) void k_resid_sum(const double *__restrict__ partials, int nb,
                                                   int nrhs, double *out) {
    const int q = blockIdx.x * (kBS / kWave) + threadIdx.x / kWave;
    if (q >= nrhs) return;
    const int lane = threadIdx.x & (kWave - 1);
    double v = 0.0;
    for (int i = lane; i < nb; i += kWave) v += partials[(int64_t)q * nb + i];
    v = wave_sum(v);
    if (lane == 0) out[q] = v;
}

// dst = src with a change of precision (grid-stride over n complex numbers)
template <typename S, typename D>
__global__ __launch_bounds__(kBS) void k_convert(const S *__restrict__ src, D *__restrict__ dst,
                                                 int64_t n) {
    using R = decltype(D{}.x);
    GRID_STRIDE(i) {
        const S v = src[i];
        dst[i] = D{(R)v.x, (R)v.y};
    }
}

// bfloat16 pairs (real part in the low half) <-> float or double
__global__ __launch_bounds__(kBS) void k_bf16_to(const uint32_t *__restrict__ src, fvec2 *__restrict__ f,
                                                 dvec2 *__restrict__ d, int64_t n) {
    GRID_STRIDE(i) {
        const uint32_t u = src[i];
        const float re = __uint_as_float(u << 16), im = __uint_as_float(u & 0xffff0000u);
        if (f) f[i] = fvec2{re, im};
        else d[i] = dvec2{(double)re, (double)im};
    }
}

// float -> bfloat16, round to nearest even
__global__ __launch_bounds__(kBS) void k_f32_to_bf16(const fvec2 *__restrict__ src,
                                                     uint32_t *__restrict__ dst, int64_t n) {
    GRID_STRIDE(i) {
        const fvec2 v = src[i];
        uint32_t a = __float_as_uint(v.x), b = __float_as_uint(v.y);
        a = (a + 0x7fffu + ((a >> 16) & 1u)) >> 16;
        b = (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
        dst[i] = a | (b << 16);
    }
}

// p = r + beta p (mode 1) or p = r (mode 2), per RHS
__global__ __launch_bounds__(kBS) void k_p_restart(fvec2 *__restrict__ p, const fvec2 *__restrict__ r,
                                                   int64_t n, const double *__restrict__ beta,
                                                   const int *__restrict__ mode) {
    const int rhs = blockIdx.y;
    const int m = mode[rhs];
    if (m == 0) return;
    const int64_t off = rhs * n;
    const float be = m == 1 ? (float)beta[rhs] : 0.0f;
    GRID_STRIDE(i) {
        const fvec2 rr = r[off + i];
        fvec2 pp = m == 1 ? p[off + i] : fvec2{0.0f, 0.0f};
        pp.x = fma(be, pp.x, rr.x);
        pp.y = fma(be, pp.y, rr.y);
        p[off + i] = pp;
    }
}

// zero the coefficient rows C[j][*] of unmasked RHS
__global__ __launch_bounds__(kBS) void k_mask_rows(dvec2 *__restrict__ C, int k, int nrhs,
                                                   const int *__restrict__ mask) {
    const int64_t e = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (e >= (int64_t)k * nrhs) return;
    const int j = (int)(e / k);
    if (!mask[j]) C[e] = dvec2{0.0, 0.0};
}

}  // namespace

#define AS_D(p) reinterpret_cast<dvec2 *>(p)
#define AS_CD(p) reinterpret_cast<const dvec2 *>(p)
#define AS_F(p) reinterpret_cast<fvec2 *>(p)
#define AS_CF(p) reinterpret_cast<const fvec2 *>(p)

hisq_status mixed_to_f32(const double2 *src, float2 *dst, int64_t n, int nrhs, const int *mask,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3(grid_x(n), nrhs), dim3(kBS), 0, s, AS_CD(src), AS_F(dst), n,
                       mask);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status convert_vectors(const void *src, hisq_prec sp, void *dst, hisq_prec dp, int64_t n,
                            hipStream_t s) {
    if (n == 0) return HISQ_OK;
    const int nb = (int)std::min<int64_t>((n + kBS - 1) / kBS, 16384);
    if (sp == HISQ_BF16 && dp != HISQ_BF16) {
        hipLaunchKernelGGL(k_bf16_to, dim3(nb), dim3(kBS), 0, s, static_cast<const uint32_t *>(src),
                           dp == HISQ_FP32 ? static_cast<fvec2 *>(dst) : nullptr,
                           dp == HISQ_FP64 ? static_cast<dvec2 *>(dst) : nullptr, n);
        HISQ_HIP(hipGetLastError());
        return HISQ_OK;
    }
    if (dp == HISQ_BF16 && sp == HISQ_FP64)
        return convert_double_to_bf16(static_cast<const double2 *>(src),
                                      static_cast<uint32_t *>(dst), n, s);
    if (dp == HISQ_BF16 && sp == HISQ_FP32) {
        hipLaunchKernelGGL(k_f32_to_bf16, dim3(nb), dim3(kBS), 0, s,
                           static_cast<const fvec2 *>(src), static_cast<uint32_t *>(dst), n);
        HISQ_HIP(hipGetLastError());
        return HISQ_OK;
    }
    if (sp == HISQ_BF16 && dp == HISQ_BF16) {
        HISQ_HIP(hipMemcpyAsync(dst, src, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        return HISQ_OK;
    }
    if (sp == HISQ_FP64 && dp == HISQ_FP32)
        hipLaunchKernelGGL((k_convert<dvec2, fvec2>), dim3(nb), dim3(kBS), 0, s,
                           static_cast<const dvec2 *>(src), static_cast<fvec2 *>(dst), n);
    else if (sp == HISQ_FP32 && dp == HISQ_FP64)
        hipLaunchKernelGGL((k_convert<fvec2, dvec2>), dim3(nb), dim3(kBS), 0, s,
                           static_cast<const fvec2 *>(src), static_cast<dvec2 *>(dst), n);
    else
        HISQ_HIP(hipMemcpyAsync(dst, src, n * (sp == HISQ_FP64 ? sizeof(double2) : sizeof(float2)),
                                hipMemcpyDeviceToDevice, s));
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status mixed_accum_x(double2 *x, float2 *xs, int64_t n, int nrhs, const int *mask,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_accum_x, dim3(grid_x(n), nrhs), dim3(kBS), 0, s, AS_D(x), AS_F(xs), n,
                       mask);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status mixed_resid(const double2 *b, const double2 *Ax, double2 *r, int64_t n, int nrhs,
                        const int *mask, double *out, const Reduce &red, hipStream_t s) {
    const int nb = grid_x(n);
    hipLaunchKernelGGL(k_resid, dim3(nb, nrhs), dim3(kBS), 0, s, AS_CD(b), AS_CD(Ax), AS_D(r), n,
                       mask, red.partials);
    const int per = kBS / kWave;
    hipLaunchKernelGGL(k_resid_sum, dim3((nrhs + per - 1) / per), dim3(kBS), 0, s, red.partials, nb,
                       nrhs, out);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

int mixed_resid_blocks(int64_t n) { return grid_x(n); }

hisq_status mixed_p_restart(float2 *p, const float2 *r, int64_t n, int nrhs, const double *beta,
                            const int *mode, hipStream_t s) {
    hipLaunchKernelGGL(k_p_restart, dim3(grid_x(n), nrhs), dim3(kBS), 0, s, AS_F(p), AS_CF(r), n,
                       beta, mode);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status mixed_mask_rows(double2 *C, int k, int nrhs, const int *mask, hipStream_t s) {
    const int64_t e = (int64_t)k * nrhs;
    hipLaunchKernelGGL(k_mask_rows, dim3((unsigned)((e + kBS - 1) / kBS)), dim3(kBS), 0, s, AS_D(C),
                       k, nrhs, mask);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

}  // namespace hisq
