// CG vector updates on 16-bit fixed-point fields (h16p: a site's three
// colours and their norm in 16 bytes; see dslash_kernel.h) for the mixed-precision CG at sloppy_prec =
// HISQ_HALF: the search direction p and A p are stored in 16 bits, the
// residual and the solution correction stay FP32, scalars and partial sums
// FP64 (the same fixed-order reductions as the FP32 and FP64 updates).
#include "dslash_kernel.h"

namespace hisq {
namespace {

constexpr int kBS = 256;
typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef double dvec2 __attribute__((ext_vector_type(2)));

// A 16-bit field is [nrhs][Vh] of h16p: three colours as int16 pairs and
// the site's norm, value = integer * norm / 32767.
__device__ __forceinline__ void load_site(const h16p *__restrict__ d, int64_t vh, int j,
                                          int64_t cb, fvec2 (&v)[3]) {
    h16c c[3];
    float n;
    h16_unpack(d[(int64_t)j * vh + cb], c, n);
    const float sc = n * (1.0f / kQ16);
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = fvec2{(float)c[k].x * sc, (float)c[k].y * sc};
}

__device__ __forceinline__ void store_site(h16p *__restrict__ d, int64_t vh, int j, int64_t cb,
                                           const fvec2 (&v)[3]) {
    float m = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) m = fmaxf(m, fmaxf(fabsf(v[k].x), fabsf(v[k].y)));
    const float qs = m > 0.0f ? kQ16 / m : 0.0f;
    h16c q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) q[k] = h16c{(short)rintf(v[k].x * qs), (short)rintf(v[k].y * qs)};
    d[(int64_t)j * vh + cb] = h16p{__builtin_bit_cast(int, q[0]), __builtin_bit_cast(int, q[1]),
                                   __builtin_bit_cast(int, q[2]), __float_as_int(m)};
}

__device__ __forceinline__ double wave_sum_partials(const double *__restrict__ p, int nb) {
    const int lane = threadIdx.x & (kWave - 1);
    double v = 0.0;
    for (int i = lane; i < nb; i += kWave) v += p[i];
    return wave_sum(v);
}

// Two consecutive sites per lane (Vh is even): one 16-byte load per site of a
// 16-bit field, one 16-byte load per colour of an FP32 field.
typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load_pair(const h16p *__restrict__ d, int64_t vh, int j,
                                          int64_t cb, fvec2 (&v)[2][3]) {
    load_site(d, vh, j, cb, v[0]);
    load_site(d, vh, j, cb + 1, v[1]);
}

__device__ __forceinline__ void store_pair(h16p *__restrict__ d, int64_t vh, int j, int64_t cb,
                                           const fvec2 (&v)[2][3]) {
    store_site(d, vh, j, cb, v[0]);
    store_site(d, vh, j, cb + 1, v[1]);
}

__device__ __forceinline__ void load_pair_f32(const fvec2 *__restrict__ f, int64_t vh, int j,
                                              int64_t cb, fvec2 (&v)[2][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const fvec4 q = *reinterpret_cast<const fvec4 *>(f + ((int64_t)j * 3 + c) * vh + cb);
        v[0][c] = fvec2{q.x, q.y};
        v[1][c] = fvec2{q.z, q.w};
    }
}

__device__ __forceinline__ void store_pair_f32(fvec2 *__restrict__ f, int64_t vh, int j, int64_t cb,
                                               const fvec2 (&v)[2][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
        *reinterpret_cast<fvec4 *>(f + ((int64_t)j * 3 + c) * vh + cb) =
            fvec4{v[0][c].x, v[0][c].y, v[1][c].x, v[1][c].y};
}

// alpha = rho / <p, Ap> (the stencil's fixed-order partials), r -= alpha Ap,
// per-block partials of ||r||^2.  Grid (blas_reduce_blocks(3 Vh), nrhs); a
// lane takes two consecutive sites at a time.  The first pair's r and A p are
// loaded before the partials are summed, so that the two memory latencies
// overlap.
__global__ __launch_bounds__(kBS) void k_update_r_h(int64_t vh, fvec2 *__restrict__ r,
                                                    const h16p *__restrict__ ap,
                                                    const double *__restrict__ pap, int nb_pap,
                                                    CgDev cg, Reduce red) {
    const int j = blockIdx.y;
    const bool active = cg.status[j] == CG_ACTIVE;
    const int64_t npair = vh / 2;
    const int64_t stride = (int64_t)gridDim.x * kBS;
    int64_t pi = (int64_t)blockIdx.x * kBS + threadIdx.x;
    fvec2 q[2][3], rr[2][3];
    if (active && pi < npair) {
        load_pair(ap, vh, j, 2 * pi, q);
        load_pair_f32(r, vh, j, 2 * pi, rr);
    }
    __shared__ double pq_s;
    if (threadIdx.x < kWave) {
        const double v = wave_sum_partials(pap + (int64_t)j * nb_pap, nb_pap);
        if (threadIdx.x == 0) pq_s = v;
    }
    __syncthreads();
    const double pq = pq_s;
    double v[1] = {0.0};
    if (active && isfinite(pq) && pq > 0.0) {
        const float al = (float)(cg.rho[j] / pq);
        while (pi < npair) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    rr[h][c].x = fmaf(-al, q[h][c].x, rr[h][c].x);
                    rr[h][c].y = fmaf(-al, q[h][c].y, rr[h][c].y);
                    v[0] = fma((double)rr[h][c].x, (double)rr[h][c].x,
                               fma((double)rr[h][c].y, (double)rr[h][c].y, v[0]));
                }
            store_pair_f32(r, vh, j, 2 * pi, rr);
            pi += stride;
            if (pi < npair) {
                load_pair(ap, vh, j, 2 * pi, q);
                load_pair_f32(r, vh, j, 2 * pi, rr);
            }
        }
    }
    __shared__ double lds[kBS / kWave];
    block_sum<1, kBS>(v, lds);
    if (threadIdx.x == 0) red.partials[(int64_t)j * gridDim.x + blockIdx.x] = v[0];
}

// x += alpha p_old; p = r + beta p_old (mode 2), or only the x update (mode 1).
// Two consecutive sites per lane; the first pair's x, p and r are loaded
// before the RHS's mode and coefficients are read.
__global__ __launch_bounds__(kBS) void k_update_xp_h(int64_t vh, fvec2 *__restrict__ x,
                                                     const fvec2 *__restrict__ r,
                                                     h16p *__restrict__ p, CgDev cg) {
    const int j = blockIdx.y;
    const int64_t npair = vh / 2;
    const int64_t stride = (int64_t)gridDim.x * kBS;
    int64_t pi = (int64_t)blockIdx.x * kBS + threadIdx.x;
    fvec2 pp[2][3], xx[2][3], rr[2][3];
    if (pi < npair) {
        load_pair(p, vh, j, 2 * pi, pp);
        load_pair_f32(x, vh, j, 2 * pi, xx);
        load_pair_f32(r, vh, j, 2 * pi, rr);
    }
    const int mode = cg.xp_mode[j];
    if (mode == 0) return;
    const float al = (float)cg.xp_alpha[j], be = (float)cg.xp_beta[j];
    while (pi < npair) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xx[h][c].x = fmaf(al, pp[h][c].x, xx[h][c].x);
                xx[h][c].y = fmaf(al, pp[h][c].y, xx[h][c].y);
                if (mode == 2)
                    pp[h][c] = fvec2{fmaf(be, pp[h][c].x, rr[h][c].x), fmaf(be, pp[h][c].y, rr[h][c].y)};
            }
        store_pair_f32(x, vh, j, 2 * pi, xx);
        if (mode == 2) store_pair(p, vh, j, 2 * pi, pp);
        pi += stride;
        if (pi < npair) {
            load_pair(p, vh, j, 2 * pi, pp);
            load_pair_f32(x, vh, j, 2 * pi, xx);
            load_pair_f32(r, vh, j, 2 * pi, rr);
        }
    }
}

// p = r + beta p (mode 1) or p = r (mode 2) per RHS; mode == null: p = r for all
__global__ __launch_bounds__(kBS) void k_p_restart_h(int64_t vh, h16p *__restrict__ p,
                                                     const fvec2 *__restrict__ r,
                                                     const double *__restrict__ beta,
                                                     const int *__restrict__ mode) {
    const int j = blockIdx.y;
    const int m = mode ? mode[j] : 2;
    if (m == 0) return;
    const float be = m == 1 ? (float)beta[j] : 0.0f;
    for (int64_t cb = (int64_t)blockIdx.x * kBS + threadIdx.x; cb < vh;
         cb += (int64_t)gridDim.x * kBS) {
        fvec2 pp[3];
        if (m == 1) load_site(p, vh, j, cb, pp);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const fvec2 rr = r[((int64_t)j * 3 + c) * vh + cb];
            pp[c] = m == 1 ? fvec2{fmaf(be, pp[c].x, rr.x), fmaf(be, pp[c].y, rr.y)} : rr;
        }
        store_site(p, vh, j, cb, pp);
    }
}

// out = the FP32 value of a 16-bit field
__global__ __launch_bounds__(kBS) void k_h16_to_f32(int64_t vh, const h16p *__restrict__ h,
                                                    fvec2 *__restrict__ out) {
    const int j = blockIdx.y;
    for (int64_t cb = (int64_t)blockIdx.x * kBS + threadIdx.x; cb < vh;
         cb += (int64_t)gridDim.x * kBS) {
        fvec2 v[3];
        load_site(h, vh, j, cb, v);
#pragma unroll
        for (int c = 0; c < 3; ++c) out[((int64_t)j * 3 + c) * vh + cb] = v[c];
    }
}

int site_blocks(int64_t vh) {
    const int64_t b = (vh + kBS - 1) / kBS;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

int64_t half_field_bytes(int64_t vh, int nrhs) { return (int64_t)nrhs * vh * (3 * 4 + 4); }

hisq_status half_update_r(int64_t vh, int nrhs, float2 *r, const void *ap, const double *pap,
                          int nb_pap, const CgDev &cg, const Reduce &red, hipStream_t s) {
    const h16p *d = static_cast<const h16p *>(ap);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_update_r_h, dim3(blas_reduce_blocks(3 * vh), nrhs), dim3(kBS), 0, s, vh,
                       reinterpret_cast<fvec2 *>(r), d, pap, nb_pap, cg, red);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status half_update_xp(int64_t vh, int nrhs, float2 *x, const float2 *r, void *p,
                           const CgDev &cg, hipStream_t s) {
    h16p *d = static_cast<h16p *>(p);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_update_xp_h, dim3(site_blocks(vh), nrhs), dim3(kBS), 0, s, vh,
                       reinterpret_cast<fvec2 *>(x), reinterpret_cast<const fvec2 *>(r), d, cg);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status half_p_restart(int64_t vh, int nrhs, void *p, const float2 *r, const double *beta,
                           const int *mode, hipStream_t s) {
    h16p *d = static_cast<h16p *>(p);
    hipLaunchKernelGGL(k_p_restart_h, dim3(site_blocks(vh), nrhs), dim3(kBS), 0, s, vh, d,
                       reinterpret_cast<const fvec2 *>(r), beta, mode);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status half_to_f32(int64_t vh, int nrhs, const void *h, float2 *out, hipStream_t s) {
    const h16p *d = static_cast<const h16p *>(h);
    hipLaunchKernelGGL(k_h16_to_f32, dim3(site_blocks(vh), nrhs), dim3(kBS), 0, s, vh, d,
                       reinterpret_cast<fvec2 *>(out));
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

// The operators at HISQ_HALF: FP32 vectors in and out, rounded to the 16-bit
// format on entry, the 16-bit stencil (as in the CG's sloppy iteration), and
// the result widened to FP32.
hisq_status apply_dslash_half(hisq_gauge_s *g, int out_parity, const float2 *in, float2 *out,
                              int nrhs, hipStream_t s) {
    const int64_t vh = g->geom.vh;
    const size_t hb = (size_t)half_field_bytes(vh, nrhs);
    void *hin = nullptr, *hout = nullptr;
    HISQ_TRY(g->ws.get("half_op_in", hb, &hin));
    HISQ_TRY(g->ws.get("half_op_out", hb, &hout));
    HISQ_TRY(half_p_restart(vh, nrhs, hin, in, nullptr, nullptr, s));
    HISQ_TRY(launch_dslash_h16(g, out_parity, hin, hout, nrhs, nullptr, 0.0, 1.0, nullptr, s));
    return half_to_f32(vh, nrhs, hout, out, s);
}

hisq_status apply_mdagm_half(hisq_gauge_s *g, double two_m, const float2 *in, float2 *out,
                             int nrhs, hipStream_t s) {
    const int64_t vh = g->geom.vh;
    const size_t hb = (size_t)half_field_bytes(vh, nrhs);
    void *hin = nullptr, *hout = nullptr, *ht = nullptr;
    HISQ_TRY(g->ws.get("half_op_in", hb, &hin));
    HISQ_TRY(g->ws.get("half_op_out", hb, &hout));
    HISQ_TRY(g->ws.get("half_op_t", hb, &ht));
    HISQ_TRY(half_p_restart(vh, nrhs, hin, in, nullptr, nullptr, s));
    HISQ_TRY(launch_dslash_h16(g, 1, hin, ht, nrhs, nullptr, 0.0, 1.0, nullptr, s));
    HISQ_TRY(launch_dslash_h16(g, 0, ht, hout, nrhs, hin, two_m * two_m, -1.0, nullptr, s));
    return half_to_f32(vh, nrhs, hout, out, s);
}

}  // namespace hisq
