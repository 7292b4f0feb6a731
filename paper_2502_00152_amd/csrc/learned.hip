// Learned initial guess: a three-layer gauge-covariant network N that maps the
// residual r0 = b - A x0 of a (deflation) initial guess to a correction of
// x0.  An extension beyond arXiv:2502.00152, whose solver is deflated CG
// (section 2): CG stays the solver, its true-residual stop is unchanged, and
// hisq_nn_guess keeps a correction only where it lowers ||b - A x||; given the
// eigenpairs, it first projects the correction off the deflation space.
//
//   layer(W, psi)^o = sum_{d=0..8} sum_c W[d][o][c] T_d psi^c
//     T_0 = 1, (T_{1+mu} psi)(x) = F_mu(x) psi(x+mu),
//     (T_{5+mu} psi)(x) = F_mu(x-mu)^H psi(x-mu)   (FP32 fat links, phases folded)
//   gate(g, psi)^c(x) = psi^c(x) sigmoid(a_c |psi^c(x)| + b_c)
//   N(r) = even part of layer(W3, gate(g2, layer(W2, gate(g1, layer(W1, r)))))
//
// Training: hand-written backward kernels.  T_{1+mu}^H = T_{5+mu}, so the
// backward data pass of a layer is the same layer kernel with the weights
// transposed over (o, c) and the two hop directions of each mu swapped.
// Activations and their gradients are FP32 (one site per lane, channels in
// registers); weight gradients, gate gradients, norms and the loss are summed
// in FP64 in a fixed order.  Adam runs on the device.
//
// Activation layout: [sample][channel][parity][colour][Vh] complex float, so
// consecutive lanes touch consecutive sites.
#include <hip/hip_bf16.h>

#include <cmath>
#include <new>
#include <vector>

#include "device_util.h"
#include "hisq_internal.h"

namespace hisq {
hisq_status check_gauge(hisq_gauge g);
hisq_status check_vec(const void *p, const char *name);
hisq_status check_nrhs(int nrhs);
hisq_status check_mass(double two_m, bool positive);
}  // namespace hisq

using namespace hisq;

namespace hisq {
namespace nn {

constexpr int C = HISQ_NN_CHANNELS;
constexpr int kBS = 256;
constexpr int OFF_W1 = 0, OFF_W2 = OFF_W1 + 9 * C, OFF_W3 = OFF_W2 + 9 * C * C,
              OFF_G1 = OFF_W3 + 9 * C, OFF_G2 = OFF_G1 + 2 * C, NPARAM = OFF_G2 + 2 * C;
static_assert(NPARAM == HISQ_NN_PARAMS, "parameter count");
constexpr int kMaxRedBlocks = 512;  // cap on the site blocks of a reduction
constexpr int kWgradBlocks = 96;    // site blocks of a weight-gradient launch: each
                                    // lane sums several sites before the 64-value
                                    // block reduction, which dominates otherwise

typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(__hip_bfloat16 v) { return __bfloat162float(v); }

// a site of the full lattice: i in [0, 2 Vh), parity i / Vh
struct Site {
    int p, cb, x, y, z, t;
};

__device__ __forceinline__ Site site_of(int i, const Geom &g) {
    Site s;
    s.p = i >= g.vh ? 1 : 0;
    s.cb = i - s.p * g.vh;
    int r = s.cb / g.Xh;
    const int xh = s.cb - r * g.Xh;
    s.y = r % g.Y;
    r /= g.Y;
    s.z = r % g.Z;
    s.t = r / g.Z;
    s.x = 2 * xh + ((s.p + s.y + s.z + s.t) & 1);
    return s;
}

__device__ __forceinline__ int wrap1(int c, int L) { return c < 0 ? c + L : (c >= L ? c - L : c); }

// checkerboard index of x + h mu, h = +-1
__device__ __forceinline__ int nb_index(const Site &s, int mu, int h, const Geom &g) {
    const int x = mu == 0 ? wrap1(s.x + h, g.X) : s.x;
    const int y = mu == 1 ? wrap1(s.y + h, g.Y) : s.y;
    const int z = mu == 2 ? wrap1(s.z + h, g.Z) : s.z;
    const int t = mu == 3 ? wrap1(s.t + h, g.T) : s.t;
    return ((((t * g.Z + z) * g.Y + y) * g.X) + x) >> 1;
}

// offset of (channel c, parity p, colour a, site cb) within one sample
__device__ __forceinline__ int64_t coff(int c, int p, int a, int cb, int vh) {
    return ((int64_t)(c * 2 + p) * 3 + a) * vh + cb;
}

__device__ __forceinline__ void load_link(const fvec2 *U, int mu, int cb, int64_t ntiles,
                                          fvec2 (&u)[9]) {
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = U[link_index(mu, k, cb, ntiles)];
}

// v = U w (DAG = false) or U^H w (DAG = true)
template <bool DAG>
__device__ __forceinline__ void mat3(const fvec2 (&u)[9], const fvec2 (&w)[3], fvec2 (&v)[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const fvec2 m = DAG ? fvec2{u[3 * b + a].x, -u[3 * b + a].y} : u[3 * a + b];
            re = fmaf(m.x, w[b].x, fmaf(-m.y, w[b].y, re));
            im = fmaf(m.x, w[b].y, fmaf(m.y, w[b].x, im));
        }
        v[a] = fvec2{re, im};
    }
}

// ------------------------------------------------------------------ layer
// out^o = sum_d sum_c W[d][o][c] T_d in^c on every site; W [9][CO][CI].
// Grid (ceil(2 Vh / 256), samples).
template <int CI, int CO, typename TW>
__global__ __launch_bounds__(kBS) void k_layer(const fvec2 *__restrict__ in, fvec2 *__restrict__ out,
                                               const TW *__restrict__ W, const fvec2 *__restrict__ fat0,
                                               const fvec2 *__restrict__ fat1, int64_t ntiles, Geom g) {
    __shared__ float w[9 * CO * CI];
    for (int e = threadIdx.x; e < 9 * CO * CI; e += kBS) w[e] = to_f(W[e]);
    __syncthreads();
    const int i = blockIdx.x * kBS + threadIdx.x;
    if (i >= 2 * g.vh) return;
    const int vh = g.vh;
    const Site st = site_of(i, g);
    const fvec2 *src = in + (int64_t)blockIdx.y * CI * 6 * vh;
    fvec2 acc[CO][3];
#pragma unroll
    for (int c = 0; c < CI; ++c) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const fvec2 v = src[coff(c, st.p, a, st.cb, vh)];
#pragma unroll
            for (int o = 0; o < CO; ++o) {
                const float wo = w[o * CI + c];
                if (c == 0) acc[o][a] = fvec2{wo * v.x, wo * v.y};
                else acc[o][a] = fvec2{fmaf(wo, v.x, acc[o][a].x), fmaf(wo, v.y, acc[o][a].y)};
            }
        }
    }
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {  // 0: T_{1+mu}, 1: T_{5+mu}
            const int nb = nb_index(st, mu, h ? -1 : 1, g);
            fvec2 u[9];
            load_link((st.p ^ h) ? fat1 : fat0, mu, h ? nb : st.cb, ntiles, u);
            const float *wd = w + (h ? 5 + mu : 1 + mu) * CO * CI;
#pragma unroll
            for (int c = 0; c < CI; ++c) {
                fvec2 x[3], v[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) x[a] = src[coff(c, 1 - st.p, a, nb, vh)];
                if (h) mat3<true>(u, x, v);
                else mat3<false>(u, x, v);
#pragma unroll
                for (int o = 0; o < CO; ++o) {
                    const float wo = wd[o * CI + c];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        acc[o][a] = fvec2{fmaf(wo, v[a].x, acc[o][a].x), fmaf(wo, v[a].y, acc[o][a].y)};
                }
            }
        }
    }
    fvec2 *dst = out + (int64_t)blockIdx.y * CO * 6 * vh;
#pragma unroll
    for (int o = 0; o < CO; ++o)
#pragma unroll
        for (int a = 0; a < 3; ++a) dst[coff(o, st.p, a, st.cb, vh)] = acc[o][a];
}

// Fixed-order block sum of NV doubles per thread, stored by thread 0 at dst.
template <int NV>
__device__ __forceinline__ void block_store_sum(double (&v)[NV], double *dst, double *lds) {
    block_sum<NV, kBS>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) dst[j] = v[j];
    }
}

// ---------------------------------------------------------- weight gradient
// dW[d][o][c] = sum_x Re<gout^o(x), (T_d in^c)(x)>.  Grid (nb, 9, S); block b
// takes sites b*256 + lane + k*nb*256; each lane sums its sites in FP32, the
// block in FP64.  Partials [d][s][b][CO*CI].
template <int CI, int CO>
__global__ __launch_bounds__(kBS) void k_wgrad(const fvec2 *__restrict__ in,
                                               const fvec2 *__restrict__ gout,
                                               const fvec2 *__restrict__ fat0,
                                               const fvec2 *__restrict__ fat1, int64_t ntiles,
                                               Geom g, double *__restrict__ partials) {
    constexpr int E = CO * CI;
    __shared__ double lds[E * (kBS / kWave)];
    const int d = blockIdx.y, s = blockIdx.z, nb = gridDim.x, S = gridDim.z, vh = g.vh;
    const fvec2 *src = in + (int64_t)s * CI * 6 * vh;
    const fvec2 *go = gout + (int64_t)s * CO * 6 * vh;
    float acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.f;
    for (int i = blockIdx.x * kBS + threadIdx.x; i < 2 * vh; i += nb * kBS) {
        const Site st = site_of(i, g);
        fvec2 gv[CO][3];
#pragma unroll
        for (int o = 0; o < CO; ++o)
#pragma unroll
            for (int a = 0; a < 3; ++a) gv[o][a] = go[coff(o, st.p, a, st.cb, vh)];
        int sp = st.p, scb = st.cb, mode = 0;  // mode 0: identity, 1: U, 2: U^H
        fvec2 u[9];
        if (d > 0) {
            const int mu = (d - 1) & 3, h = d > 4;
            const int nbi = nb_index(st, mu, h ? -1 : 1, g);
            load_link((st.p ^ h) ? fat1 : fat0, mu, h ? nbi : st.cb, ntiles, u);
            sp = 1 - st.p;
            scb = nbi;
            mode = 1 + h;
        }
#pragma unroll
        for (int c = 0; c < CI; ++c) {
            fvec2 x[3], v[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) x[a] = src[coff(c, sp, a, scb, vh)];
            if (mode == 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) v[a] = x[a];
            } else if (mode == 1) {
                mat3<false>(u, x, v);
            } else {
                mat3<true>(u, x, v);
            }
#pragma unroll
            for (int o = 0; o < CO; ++o) {
                float t = acc[o * CI + c];
#pragma unroll
                for (int a = 0; a < 3; ++a) t = fmaf(gv[o][a].x, v[a].x, fmaf(gv[o][a].y, v[a].y, t));
                acc[o * CI + c] = t;
            }
        }
    }
    double v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = acc[e];
    block_store_sum<E>(v, partials + (((int64_t)d * S + s) * nb + blockIdx.x) * E, lds);
}

__device__ __forceinline__ float sigm(float u) { return 1.f / (1.f + __expf(-u)); }

// ------------------------------------------------------------------- gates
// y = z sigmoid(a |z| + b) per site and channel (y may equal z); ab [C][2].
// Grid (ceil(2 Vh / 256), C, S).
template <typename TW>
__global__ __launch_bounds__(kBS) void k_gate(const fvec2 *z, fvec2 *y, const TW *__restrict__ ab,
                                              int vh) {
    const int i = blockIdx.x * kBS + threadIdx.x, c = blockIdx.y, s = blockIdx.z;
    if (i >= 2 * vh) return;
    const int p = i >= vh, cb = i - p * vh;
    const int64_t base = (int64_t)s * C * 6 * vh;
    fvec2 v[3];
    float n2 = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v[a] = z[base + coff(c, p, a, cb, vh)];
        n2 = fmaf(v[a].x, v[a].x, fmaf(v[a].y, v[a].y, n2));
    }
    const float sg = sigm(to_f(ab[2 * c]) * sqrtf(n2) + to_f(ab[2 * c + 1]));
#pragma unroll
    for (int a = 0; a < 3; ++a) y[base + coff(c, p, a, cb, vh)] = fvec2{v[a].x * sg, v[a].y * sg};
}

// Backward of the gate: gz = s gy + (Re<gy, z> s (1 - s) a / |z|) z, and block
// partials of dL/da_c = sum Re<gy, z> s (1 - s) |z|, dL/db_c = sum Re<gy, z>
// s (1 - s).  Grid (nb, C, S), lanes loop over sites; partials [c][s][b][2].
__global__ __launch_bounds__(kBS) void k_gate_bwd(const fvec2 *__restrict__ z,
                                                  const fvec2 *__restrict__ gy,
                                                  fvec2 *__restrict__ gz,
                                                  const float *__restrict__ ab, int vh,
                                                  double *__restrict__ partials) {
    __shared__ double lds[2 * (kBS / kWave)];
    const int c = blockIdx.y, s = blockIdx.z, nb = gridDim.x, S = gridDim.z;
    const int64_t base = (int64_t)s * C * 6 * vh;
    const float av = ab[2 * c], bv = ab[2 * c + 1];
    float pa = 0.f, pb = 0.f;
    for (int i = blockIdx.x * kBS + threadIdx.x; i < 2 * vh; i += nb * kBS) {
        const int p = i >= vh, cb = i - p * vh;
        fvec2 v[3], g[3];
        float n2 = 0.f, dot = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = z[base + coff(c, p, a, cb, vh)];
            g[a] = gy[base + coff(c, p, a, cb, vh)];
            n2 = fmaf(v[a].x, v[a].x, fmaf(v[a].y, v[a].y, n2));
            dot = fmaf(g[a].x, v[a].x, fmaf(g[a].y, v[a].y, dot));
        }
        const float n = sqrtf(n2);
        const float sg = sigm(av * n + bv);
        const float ds = dot * sg * (1.f - sg);
        const float k = n > 0.f ? ds * av / n : 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            gz[base + coff(c, p, a, cb, vh)] =
                fvec2{fmaf(g[a].x, sg, v[a].x * k), fmaf(g[a].y, sg, v[a].y * k)};
        pa = fmaf(ds, n, pa);
        pb += ds;
    }
    double v[2] = {pa, pb};
    block_store_sum<2>(v, partials + (((int64_t)c * S + s) * nb + blockIdx.x) * 2, lds);
}

// ------------------------------------------------- input, loss and output
// Per-sample block partials of ||r_s||^2 and ||e_s||^2 (e may be null).
// Grid (nb, S); partials [s][b][2].
__global__ __launch_bounds__(kBS) void k_norms(const dvec2 *__restrict__ r, const dvec2 *__restrict__ e,
                                               int vh, double *__restrict__ partials) {
    __shared__ double lds[2 * (kBS / kWave)];
    const int s = blockIdx.y, nb = gridDim.x;
    const int64_t n = 3 * (int64_t)vh;
    double v[2] = {0.0, 0.0};
    for (int64_t k = (int64_t)blockIdx.x * kBS + threadIdx.x; k < n; k += (int64_t)nb * kBS) {
        const dvec2 a = r[s * n + k];
        v[0] = fma(a.x, a.x, fma(a.y, a.y, v[0]));
        if (e) {
            const dvec2 b = e[s * n + k];
            v[1] = fma(b.x, b.x, fma(b.y, b.y, v[1]));
        }
    }
    block_store_sum<2>(v, partials + ((int64_t)s * nb + blockIdx.x) * 2, lds);
}

// out[j] = sum_k partials[(j / E) * dstride + (j % E) + k * E], k < nk: one
// wave per j, fixed order.
__global__ __launch_bounds__(kBS) void k_sum(const double *__restrict__ partials, int nj, int E,
                                             int64_t dstride, int64_t nk, double *__restrict__ out) {
    const int j = blockIdx.x * (kBS / kWave) + threadIdx.x / kWave;
    if (j >= nj) return;
    const int lane = threadIdx.x & (kWave - 1);
    const double *p = partials + (int64_t)(j / E) * dstride + (j % E);
    double v = 0.0;
    for (int64_t k = lane; k < nk; k += kWave) v += p[k * E];
    v = wave_sum(v);
    if (lane == 0) out[j] = v;
}

// act0 (one channel): even sites = scale_s r_s, odd sites 0; scale_s =
// 1/||r_s|| with normalisation (0 for r_s = 0), else 1.  Grid (nb, S).
__global__ __launch_bounds__(kBS) void k_input(const dvec2 *__restrict__ r, fvec2 *__restrict__ act,
                                               const double *__restrict__ norms, int normalize,
                                               int vh) {
    const int s = blockIdx.y;
    const double n2 = norms[2 * s];
    const double sc = normalize ? (n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0) : 1.0;
    const int64_t n = 3 * (int64_t)vh;
    fvec2 *dst = act + (int64_t)s * 6 * vh;
    for (int64_t k = (int64_t)blockIdx.x * kBS + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBS) {
        const dvec2 v = r[s * n + k];
        dst[k] = fvec2{(float)(v.x * sc), (float)(v.y * sc)};  // parity 0 block: [3][Vh]
        dst[n + k] = fvec2{0.f, 0.f};                            // parity 1 block
    }
}

// dz3 = z3_even - scale_s e_s; gz3 = 2 dz3 / (S ||scale_s e_s||^2) on even
// sites, 0 on odd ones; block partials of ||dz3||^2 / (S ||scale_s e_s||^2).
// Grid (nb, S); partials [s][b].
__global__ __launch_bounds__(kBS) void k_loss(const fvec2 *__restrict__ z3, const dvec2 *__restrict__ e,
                                              const double *__restrict__ norms, int normalize,
                                              int vh, fvec2 *__restrict__ gz3,
                                              double *__restrict__ partials) {
    __shared__ double lds[kBS / kWave];
    const int s = blockIdx.y, nb = gridDim.x, S = gridDim.y;
    const double r2 = norms[2 * s];
    const double sc = normalize ? (r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0) : 1.0;
    const double w = 1.0 / (S * norms[2 * s + 1] * sc * sc);
    const int64_t n = 3 * (int64_t)vh;
    const fvec2 *zs = z3 + (int64_t)s * 6 * vh;
    fvec2 *gs = gz3 + (int64_t)s * 6 * vh;
    double v[1] = {0.0};
    for (int64_t k = (int64_t)blockIdx.x * kBS + threadIdx.x; k < n; k += (int64_t)nb * kBS) {
        const fvec2 o = zs[k];
        const dvec2 t = e[s * n + k];
        const double dx = (double)o.x - t.x * sc, dy = (double)o.y - t.y * sc;
        v[0] = fma(dx, dx, fma(dy, dy, v[0]));
        gs[k] = fvec2{(float)(2.0 * w * dx), (float)(2.0 * w * dy)};
        gs[n + k] = fvec2{0.f, 0.f};
    }
    v[0] *= w;
    block_store_sum<1>(v, partials + (int64_t)s * nb + blockIdx.x, lds);
}

// out_s = z3_even / scale_s (complex double).  Grid (nb, S).
__global__ __launch_bounds__(kBS) void k_output(const fvec2 *__restrict__ z3, dvec2 *__restrict__ out,
                                                const double *__restrict__ norms, int normalize,
                                                int vh) {
    const int s = blockIdx.y;
    const double sc = normalize ? sqrt(norms[2 * s]) : 1.0;
    const int64_t n = 3 * (int64_t)vh;
    const fvec2 *zs = z3 + (int64_t)s * 6 * vh;
    for (int64_t k = (int64_t)blockIdx.x * kBS + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBS) {
        const fvec2 o = zs[k];
        out[s * n + k] = dvec2{o.x * sc, o.y * sc};
    }
}

// -------------------------------------------------------- parameter kernels
// Weights of the backward data pass: WT[adj(d)][c][o] = W[d][o][c] with
// adj(0) = 0, adj(1+mu) = 5+mu, adj(5+mu) = 1+mu.
__global__ void k_transpose(const float *__restrict__ W, float *__restrict__ WT, int co, int ci) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * co * ci) return;
    const int d = e / (co * ci), rem = e - d * co * ci, o = rem / ci, c = rem - o * ci;
    const int da = d == 0 ? 0 : (d <= 4 ? d + 4 : d - 4);
    WT[(da * ci + c) * co + o] = W[e];
}

// Adam (Kingma and Ba 2015): m, v moments, bias corrections c1 = 1 - beta1^t,
// c2 = 1 - beta2^t.
__global__ void k_adam(float *__restrict__ theta, const double *__restrict__ grad,
                       float *__restrict__ m, float *__restrict__ v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = (float)grad[k];
    const float mk = fmaf(b1, m[k], (1.f - b1) * gk);
    const float vk = fmaf(b2, v[k], (1.f - b2) * gk * gk);
    m[k] = mk;
    v[k] = vk;
    theta[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void k_to_bf16(const float *__restrict__ a, __hip_bfloat16 *__restrict__ b, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) b[k] = __float2bfloat16(a[k]);  // round to nearest even
}

// keep[j] = ||r'_j||^2 < ||r_j||^2; x_j += d_j where kept.  Grid (nb, nrhs).
__global__ __launch_bounds__(kBS) void k_keep_add(dvec2 *__restrict__ x, const dvec2 *__restrict__ d,
                                                  const double *__restrict__ r2_old,
                                                  const double *__restrict__ r2_new,
                                                  int *__restrict__ keep, int64_t n) {
    const int j = blockIdx.y;
    const bool k = r2_new[j] < r2_old[j];
    if (blockIdx.x == 0 && threadIdx.x == 0) keep[j] = k ? 1 : 0;
    if (!k) return;
    for (int64_t q = (int64_t)blockIdx.x * kBS + threadIdx.x; q < n; q += (int64_t)gridDim.x * kBS)
        x[j * n + q] += d[j * n + q];
}

// y += x (complex double)
__global__ __launch_bounds__(kBS) void k_axpy(dvec2 *__restrict__ y, const dvec2 *__restrict__ x,
                                              int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * kBS + threadIdx.x; q < n; q += (int64_t)gridDim.x * kBS)
        y[q] += x[q];
}

int blocks_for(int64_t n, int cap) {
    const int64_t b = (n + kBS - 1) / kBS;
    return (int)(b < cap ? (b < 1 ? 1 : b) : cap);
}

}  // namespace nn
}  // namespace hisq

using namespace hisq::nn;

// The network handle: parameters, transposed weights, gradient and Adam
// moments in one device block; activations in a workspace.
struct hisq_nn_s {
    hisq_gauge_s *g = nullptr;
    void *block = nullptr;
    float *theta = nullptr;            // [752]
    __hip_bfloat16 *theta_bf = nullptr;  // [752], rounded copy of theta
    float *wt2 = nullptr;              // W2 transposed [9][8][8]
    float *wt3 = nullptr;              // W3 transposed [9][8][1]
    double *grad = nullptr;            // [752]
    float *m = nullptr, *v = nullptr;  // Adam moments [752]
    double *scal = nullptr;            // [1]: the loss of the last batch
    bool bf_stale = true;
    bool have_grad = false;
    int t = 0;                         // Adam steps taken
    hisq::Workspace ws;
};

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

hisq_status check_nn(hisq_nn n) {
    if (!n) return fail(HISQ_ERR_INVALID_ARG, "null network handle");
    return check_gauge(n->g);
}

hisq_status check_flags(unsigned flags) {
    if (flags & ~(unsigned)(HISQ_NN_NORMALIZE | HISQ_NN_BF16))
        return fail(HISQ_ERR_INVALID_ARG, "unknown network flag");
    return HISQ_OK;
}

hisq_status check_samples(int nsamp) {
    if (nsamp < 1 || nsamp > 4096) return fail(HISQ_ERR_INVALID_ARG, "sample count out of range");
    return HISQ_OK;
}

hisq_status ws_get(hisq_nn n, const char *name, size_t bytes, void **p) {
    return n->ws.get(name, bytes, p);
}

// one complex-float field of C channels for S samples
size_t act_bytes(const Geom &g, int S, int ch) { return sizeof(fvec2) * 6 * (size_t)g.vh * ch * S; }

template <int CI, int CO, typename TW>
hisq_status layer(hisq_nn n, const fvec2 *in, fvec2 *out, const TW *W, int S, hipStream_t s) {
    const Geom &g = n->g->geom;
    ProfileScope prof("nn_layer", s);
    hipLaunchKernelGGL((k_layer<CI, CO, TW>), dim3((2 * g.vh + kBS - 1) / kBS, S), dim3(kBS), 0, s,
                       in, out, W, reinterpret_cast<const fvec2 *>(n->g->fat32[0]),
                       reinterpret_cast<const fvec2 *>(n->g->fat32[1]), link_tiles(g.vh), g);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

template <typename TW>
hisq_status gate(hisq_nn n, const fvec2 *z, fvec2 *y, const TW *ab, int S, hipStream_t s) {
    const Geom &g = n->g->geom;
    hipLaunchKernelGGL((k_gate<TW>), dim3((2 * g.vh + kBS - 1) / kBS, C, S), dim3(kBS), 0, s, z, y, ab,
                       g.vh);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status sum(const double *partials, int nj, int E, int64_t dstride, int64_t nk, double *out,
                hipStream_t s) {
    const int per = kBS / kWave;
    hipLaunchKernelGGL(k_sum, dim3((nj + per - 1) / per), dim3(kBS), 0, s, partials, nj, E, dstride,
                       nk, out);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

// per-sample ||r||^2, ||e||^2 into norms [S][2]
hisq_status norms(hisq_nn n, const dvec2 *r, const dvec2 *e, int S, double *partials,
                  double *out, hipStream_t s) {
    const int vh = n->g->geom.vh;
    const int nb = blocks_for(3 * (int64_t)vh, kMaxRedBlocks);
    hipLaunchKernelGGL(k_norms, dim3(nb, S), dim3(kBS), 0, s, r, e, vh, partials);
    HISQ_HIP(hipGetLastError());
    return sum(partials, 2 * S, 2, 2 * (int64_t)nb, nb, out, s);
}

hisq_status refresh_bf16(hisq_nn n, hipStream_t s) {
    if (!n->bf_stale) return HISQ_OK;
    hipLaunchKernelGGL(k_to_bf16, dim3((NPARAM + kBS - 1) / kBS), dim3(kBS), 0, s, n->theta,
                       n->theta_bf, NPARAM);
    HISQ_HIP(hipGetLastError());
    n->bf_stale = false;
    return HISQ_OK;
}

// Forward pass over S samples.  Training keeps every activation (a0, z1, a1,
// z2, a2, z3); inference gates in place and reuses buffers.
struct Acts {
    fvec2 *a0, *z1, *a1, *z2, *a2, *z3;
    double *norms, *partials;
};

hisq_status get_acts(hisq_nn n, int S, bool train, Acts &A) {
    const Geom &g = n->g->geom;
    void *p = nullptr;
    HISQ_TRY(ws_get(n, "a0", act_bytes(g, S, 1), &p));
    A.a0 = static_cast<fvec2 *>(p);
    HISQ_TRY(ws_get(n, "z1", act_bytes(g, S, C), &p));
    A.z1 = static_cast<fvec2 *>(p);
    HISQ_TRY(ws_get(n, "z2", act_bytes(g, S, C), &p));
    A.z2 = static_cast<fvec2 *>(p);
    if (train) {
        HISQ_TRY(ws_get(n, "a1", act_bytes(g, S, C), &p));
        A.a1 = static_cast<fvec2 *>(p);
        HISQ_TRY(ws_get(n, "a2", act_bytes(g, S, C), &p));
        A.a2 = static_cast<fvec2 *>(p);
        HISQ_TRY(ws_get(n, "z3", act_bytes(g, S, 1), &p));
        A.z3 = static_cast<fvec2 *>(p);
    } else {
        A.a1 = A.z1;
        A.a2 = A.z2;
        A.z3 = A.a0;
    }
    HISQ_TRY(ws_get(n, "norms", sizeof(double) * 2 * (size_t)S, &p));
    A.norms = static_cast<double *>(p);
    const int nbw = blocks_for(2 * (int64_t)g.vh, kMaxRedBlocks);
    const size_t pw = (size_t)9 * S * nbw * C * C;             // weight-gradient partials
    const size_t pn = (size_t)2 * S * kMaxRedBlocks;           // norms, loss, gates
    HISQ_TRY(ws_get(n, "partials", sizeof(double) * (pw > pn * C ? pw : pn * C), &p));
    A.partials = static_cast<double *>(p);
    return HISQ_OK;
}

template <typename TW>
hisq_status forward(hisq_nn n, const TW *th, const dvec2 *r, const dvec2 *e, int S, bool normalize,
                    Acts &A, hipStream_t s) {
    const int vh = n->g->geom.vh;
    HISQ_TRY(norms(n, r, e, S, A.partials, A.norms, s));
    hipLaunchKernelGGL(k_input, dim3(blocks_for(3 * (int64_t)vh, 4096), S), dim3(kBS), 0, s, r, A.a0,
                       A.norms, normalize ? 1 : 0, vh);
    HISQ_HIP(hipGetLastError());
    HISQ_TRY((layer<1, C, TW>(n, A.a0, A.z1, th + OFF_W1, S, s)));
    HISQ_TRY(gate<TW>(n, A.z1, A.a1, th + OFF_G1, S, s));
    HISQ_TRY((layer<C, C, TW>(n, A.a1, A.z2, th + OFF_W2, S, s)));
    HISQ_TRY(gate<TW>(n, A.z2, A.a2, th + OFF_G2, S, s));
    return layer<C, 1, TW>(n, A.a2, A.z3, th + OFF_W3, S, s);
}

hisq_status apply_net(hisq_nn n, const dvec2 *r, dvec2 *out, int S, unsigned flags, hipStream_t s) {
    HISQ_TRY(ensure_links_f32(n->g, s));
    Acts A{};
    HISQ_TRY(get_acts(n, S, false, A));
    const bool norm = flags & HISQ_NN_NORMALIZE;
    if (flags & HISQ_NN_BF16) {
        HISQ_TRY(refresh_bf16(n, s));
        HISQ_TRY(forward(n, (const __hip_bfloat16 *)n->theta_bf, r, nullptr, S, norm, A, s));
    } else {
        HISQ_TRY(forward(n, (const float *)n->theta, r, nullptr, S, norm, A, s));
    }
    const int vh = n->g->geom.vh;
    hipLaunchKernelGGL(k_output, dim3(blocks_for(3 * (int64_t)vh, 4096), S), dim3(kBS), 0, s, A.z3,
                       out, A.norms, norm ? 1 : 0, vh);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

template <int CI, int CO>
hisq_status wgrad(hisq_nn n, const fvec2 *in, const fvec2 *gout, int S, double *partials,
                  double *out, hipStream_t s) {
    const Geom &g = n->g->geom;
    const int nb = blocks_for(2 * (int64_t)g.vh, kWgradBlocks);
    hipLaunchKernelGGL((k_wgrad<CI, CO>), dim3(nb, 9, S), dim3(kBS), 0, s, in, gout,
                       reinterpret_cast<const fvec2 *>(n->g->fat32[0]),
                       reinterpret_cast<const fvec2 *>(n->g->fat32[1]), link_tiles(g.vh), g,
                       partials);
    HISQ_HIP(hipGetLastError());
    constexpr int E = CO * CI;
    return sum(partials, 9 * E, E, (int64_t)S * nb * E, (int64_t)S * nb, out, s);
}

hisq_status gate_bwd(hisq_nn n, const fvec2 *z, const fvec2 *gy, fvec2 *gz, const float *ab, int S,
                     double *partials, double *out, hipStream_t s) {
    const int vh = n->g->geom.vh;
    const int nb = blocks_for(2 * (int64_t)vh, kMaxRedBlocks);
    hipLaunchKernelGGL(k_gate_bwd, dim3(nb, C, S), dim3(kBS), 0, s, z, gy, gz, ab, vh, partials);
    HISQ_HIP(hipGetLastError());
    return sum(partials, 2 * C, 2, (int64_t)S * nb * 2, (int64_t)S * nb, out, s);
}

// loss of the batch into n->scal[0] and its gradient into n->grad
hisq_status loss_grad(hisq_nn n, const dvec2 *r, const dvec2 *e, int S, unsigned flags,
                      hipStream_t s) {
    HISQ_TRY(ensure_links_f32(n->g, s));
    const Geom &g = n->g->geom;
    const int vh = g.vh;
    const bool norm = flags & HISQ_NN_NORMALIZE;
    Acts A{};
    HISQ_TRY(get_acts(n, S, true, A));
    void *p = nullptr;
    HISQ_TRY(ws_get(n, "g3", act_bytes(g, S, 1), &p));
    fvec2 *gz3 = static_cast<fvec2 *>(p);
    HISQ_TRY(ws_get(n, "ga", act_bytes(g, S, C), &p));
    fvec2 *ga = static_cast<fvec2 *>(p);
    HISQ_TRY(ws_get(n, "gz", act_bytes(g, S, C), &p));
    fvec2 *gz = static_cast<fvec2 *>(p);

    HISQ_TRY(forward(n, (const float *)n->theta, r, e, S, norm, A, s));
    const int nbl = blocks_for(3 * (int64_t)vh, kMaxRedBlocks);
    hipLaunchKernelGGL(k_loss, dim3(nbl, S), dim3(kBS), 0, s, A.z3, e, A.norms, norm ? 1 : 0, vh,
                       gz3, A.partials);
    HISQ_HIP(hipGetLastError());
    HISQ_TRY(sum(A.partials, 1, 1, 0, (int64_t)S * nbl, n->scal, s));

    hipLaunchKernelGGL(k_transpose, dim3(3), dim3(kBS), 0, s, n->theta + OFF_W2, n->wt2, C, C);
    hipLaunchKernelGGL(k_transpose, dim3(1), dim3(kBS), 0, s, n->theta + OFF_W3, n->wt3, 1, C);
    HISQ_HIP(hipGetLastError());
    // layer 3
    HISQ_TRY((wgrad<C, 1>(n, A.a2, gz3, S, A.partials, n->grad + OFF_W3, s)));
    HISQ_TRY((layer<1, C, float>(n, gz3, ga, n->wt3, S, s)));
    // gate 2, layer 2
    HISQ_TRY(gate_bwd(n, A.z2, ga, gz, n->theta + OFF_G2, S, A.partials, n->grad + OFF_G2, s));
    HISQ_TRY((wgrad<C, C>(n, A.a1, gz, S, A.partials, n->grad + OFF_W2, s)));
    HISQ_TRY((layer<C, C, float>(n, gz, ga, n->wt2, S, s)));
    // gate 1, layer 1 (gz is free again once layer 2's backward has read it)
    HISQ_TRY(gate_bwd(n, A.z1, ga, gz, n->theta + OFF_G1, S, A.partials, n->grad + OFF_G1, s));
    HISQ_TRY((wgrad<1, C>(n, A.a0, gz, S, A.partials, n->grad + OFF_W1, s)));
    n->have_grad = true;
    return HISQ_OK;
}

hisq_status adam(hisq_nn n, double lr, double b1, double b2, double eps, hipStream_t s) {
    if (!n->have_grad) return fail(HISQ_ERR_INVALID_ARG, "no gradient computed yet");
    if (!(lr > 0.0) || !std::isfinite(lr) || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) ||
        !(eps > 0.0) || !std::isfinite(eps))
        return fail(HISQ_ERR_INVALID_ARG, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
    n->t += 1;
    const double c1 = 1.0 - std::pow(b1, n->t), c2 = 1.0 - std::pow(b2, n->t);
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + kBS - 1) / kBS), dim3(kBS), 0, s, n->theta, n->grad,
                       n->m, n->v, NPARAM, (float)lr, (float)b1, (float)b2, (float)eps, (float)c1,
                       (float)c2);
    HISQ_HIP(hipGetLastError());
    n->bf_stale = true;
    return HISQ_OK;
}

hisq_status upload(hisq_nn n, const float *params_host) {
    const size_t pb = sizeof(float) * NPARAM;
    if (params_host) {
        for (int k = 0; k < NPARAM; ++k)
            if (!std::isfinite(params_host[k]))
                return fail(HISQ_ERR_INVALID_ARG, "network parameters must be finite");
        HISQ_HIP(hipMemcpy(n->theta, params_host, pb, hipMemcpyHostToDevice));
    } else {
        HISQ_HIP(hipMemset(n->theta, 0, pb));
    }
    HISQ_HIP(hipMemset(n->m, 0, pb));
    HISQ_HIP(hipMemset(n->v, 0, pb));
    // the clears go to the null stream: complete them before any caller's
    // stream can read these arrays
    HISQ_HIP(hipDeviceSynchronize());
    n->t = 0;
    n->have_grad = false;
    n->bf_stale = true;
    return HISQ_OK;
}

hisq_status check_pair_overlap(const void *a, const void *b, size_t bytes, const char *what) {
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    if (x < y + bytes && y < x + bytes) return fail(HISQ_ERR_INVALID_ARG, what);
    return HISQ_OK;
}

}  // namespace

extern "C" {

hisq_status hisq_nn_create(hisq_nn *out, hisq_gauge g, const float *params_host) {
    if (!out) return fail(HISQ_ERR_INVALID_ARG, "hisq_nn_create: null out");
    *out = nullptr;
    HISQ_TRY(check_gauge(g));
    hisq_nn n = new (std::nothrow) hisq_nn_s;
    if (!n) return fail(HISQ_ERR_OOM, "hisq_nn_create: host allocation failed");
    n->g = g;
    const size_t fb = up(sizeof(float) * NPARAM), bb = up(sizeof(__hip_bfloat16) * NPARAM),
                 db = up(sizeof(double) * NPARAM);
    const size_t total = 3 * fb + bb + up(sizeof(float) * 9 * C * C) + up(sizeof(float) * 9 * C) + db +
                         up(sizeof(double));
    if (hipMalloc(&n->block, total) != hipSuccess) {
        delete n;
        return fail(HISQ_ERR_OOM, "hisq_nn_create: device allocation failed");
    }
    char *p = static_cast<char *>(n->block);
    n->theta = reinterpret_cast<float *>(p);
    p += fb;
    n->m = reinterpret_cast<float *>(p);
    p += fb;
    n->v = reinterpret_cast<float *>(p);
    p += fb;
    n->theta_bf = reinterpret_cast<__hip_bfloat16 *>(p);
    p += bb;
    n->wt2 = reinterpret_cast<float *>(p);
    p += up(sizeof(float) * 9 * C * C);
    n->wt3 = reinterpret_cast<float *>(p);
    p += up(sizeof(float) * 9 * C);
    n->grad = reinterpret_cast<double *>(p);
    p += db;
    n->scal = reinterpret_cast<double *>(p);
    const hisq_status st = upload(n, params_host);
    if (st != HISQ_OK) {
        (void)hipFree(n->block);
        delete n;
        return st;
    }
    *out = n;
    return HISQ_OK;
}

hisq_status hisq_nn_destroy(hisq_nn n) {
    if (!n) return HISQ_OK;
    HISQ_TRY(check_gauge(n->g));
    HISQ_HIP(hipDeviceSynchronize());
    n->ws.release();
    (void)hipFree(n->block);
    delete n;
    return HISQ_OK;
}

hisq_status hisq_nn_set_params(hisq_nn n, const float *params_host) {
    HISQ_TRY(check_nn(n));
    if (!params_host) return fail(HISQ_ERR_INVALID_ARG, "params_host is null");
    HISQ_HIP(hipDeviceSynchronize());
    return upload(n, params_host);
}

hisq_status hisq_nn_get_params(hisq_nn n, float *params_host) {
    HISQ_TRY(check_nn(n));
    if (!params_host) return fail(HISQ_ERR_INVALID_ARG, "params_host is null");
    HISQ_HIP(hipDeviceSynchronize());
    HISQ_HIP(hipMemcpy(params_host, n->theta, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    return HISQ_OK;
}

hisq_status hisq_nn_apply(hisq_nn n, const void *r_dev, void *out_dev, int nsamp, unsigned flags,
                          void *stream) {
    HISQ_TRY(check_nn(n));
    HISQ_TRY(check_samples(nsamp));
    HISQ_TRY(check_flags(flags));
    HISQ_TRY(check_vec(r_dev, "r_dev"));
    HISQ_TRY(check_vec(out_dev, "out_dev"));
    const size_t vb = sizeof(double2) * 3 * (size_t)n->g->geom.vh * nsamp;
    HISQ_TRY(check_pair_overlap(r_dev, out_dev, vb, "r and out must not overlap"));
    return apply_net(n, static_cast<const dvec2 *>(r_dev), static_cast<dvec2 *>(out_dev), nsamp,
                     flags, static_cast<hipStream_t>(stream));
}

hisq_status hisq_nn_loss_grad(hisq_nn n, const void *r_dev, const void *e_dev, int nsamp,
                              unsigned flags, double *loss_host, double *grad_host, void *stream) {
    HISQ_TRY(check_nn(n));
    HISQ_TRY(check_samples(nsamp));
    HISQ_TRY(check_flags(flags));
    if (flags & HISQ_NN_BF16) return fail(HISQ_ERR_INVALID_ARG, "training runs in FP32: no BF16 flag");
    HISQ_TRY(check_vec(r_dev, "r_dev"));
    HISQ_TRY(check_vec(e_dev, "e_dev"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    HISQ_TRY(loss_grad(n, static_cast<const dvec2 *>(r_dev), static_cast<const dvec2 *>(e_dev), nsamp,
                       flags, s));
    double loss = 0.0;
    HISQ_HIP(hipMemcpyAsync(&loss, n->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad_host)
        HISQ_HIP(hipMemcpyAsync(grad_host, n->grad, sizeof(double) * NPARAM, hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(loss)) return fail(HISQ_ERR_NAN, "network loss is not finite (e_s = 0?)");
    if (loss_host) *loss_host = loss;
    return HISQ_OK;
}

hisq_status hisq_nn_adam_step(hisq_nn n, double lr, double beta1, double beta2, double eps,
                              void *stream) {
    HISQ_TRY(check_nn(n));
    return adam(n, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream));
}

hisq_status hisq_nn_train(hisq_nn n, const void *r_dev, const void *e_dev, int npairs, int batch,
                          int steps, double lr, unsigned flags, double *loss_host, void *stream) {
    HISQ_TRY(check_nn(n));
    HISQ_TRY(check_flags(flags));
    if (flags & HISQ_NN_BF16) return fail(HISQ_ERR_INVALID_ARG, "training runs in FP32: no BF16 flag");
    HISQ_TRY(check_samples(batch));
    if (npairs < batch) return fail(HISQ_ERR_INVALID_ARG, "npairs must be >= batch");
    if (steps < 0) return fail(HISQ_ERR_INVALID_ARG, "steps must be >= 0");
    HISQ_TRY(check_vec(r_dev, "r_dev"));
    HISQ_TRY(check_vec(e_dev, "e_dev"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n3 = 3 * (int64_t)n->g->geom.vh;
    const int nbatches = npairs / batch;
    void *p = nullptr;
    HISQ_TRY(ws_get(n, "losses", sizeof(double) * (size_t)(steps > 0 ? steps : 1), &p));
    double *d_losses = static_cast<double *>(p);
    for (int k = 0; k < steps; ++k) {
        const int64_t off = (int64_t)(k % nbatches) * batch * n3;
        HISQ_TRY(loss_grad(n, static_cast<const dvec2 *>(r_dev) + off,
                           static_cast<const dvec2 *>(e_dev) + off, batch, flags, s));
        HISQ_HIP(hipMemcpyAsync(d_losses + k, n->scal, sizeof(double), hipMemcpyDeviceToDevice, s));
        HISQ_TRY(adam(n, lr, 0.9, 0.999, 1e-8, s));
    }
    if (loss_host && steps > 0)
        HISQ_HIP(hipMemcpyAsync(loss_host, d_losses, sizeof(double) * steps, hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    if (loss_host)
        for (int k = 0; k < steps; ++k)
            if (!std::isfinite(loss_host[k])) return fail(HISQ_ERR_NAN, "network loss is not finite");
    return HISQ_OK;
}

hisq_status hisq_nn_guess(hisq_nn n, double two_m, const void *b_dev, void *x_dev, int nrhs,
                          unsigned flags, int n_ev, const void *evecs_dev, hisq_prec evec_prec,
                          const double *evals_host, int *kept_host, void *stream) {
    HISQ_TRY(check_nn(n));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_mass(two_m, true));
    HISQ_TRY(check_flags(flags));
    HISQ_TRY(check_vec(b_dev, "b_dev"));
    HISQ_TRY(check_vec(x_dev, "x_dev"));
    hisq_gauge_s *g = n->g;
    const int64_t n3 = 3 * (int64_t)g->geom.vh;
    const size_t vb = sizeof(double2) * (size_t)n3 * nrhs;
    HISQ_TRY(check_pair_overlap(b_dev, x_dev, vb, "b and x must not overlap"));
    if (n_ev < 0) return fail(HISQ_ERR_INVALID_ARG, "n_ev must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *p = nullptr;
    HISQ_TRY(ws_get(n, "guess_t", vb, &p));
    double2 *t = static_cast<double2 *>(p);
    HISQ_TRY(ws_get(n, "guess_r", vb, &p));
    double2 *r = static_cast<double2 *>(p);
    HISQ_TRY(ws_get(n, "guess_d", vb, &p));
    double2 *d = static_cast<double2 *>(p);
    HISQ_TRY(ws_get(n, "guess_r2", sizeof(double) * 2 * (size_t)nrhs + sizeof(int) * (size_t)nrhs, &p));
    double *r2 = static_cast<double *>(p);
    int *keep = reinterpret_cast<int *>(r2 + 2 * nrhs);
    Reduce red{};
    HISQ_TRY(ws_get(n, "guess_partials", sizeof(double) * (size_t)nrhs * mixed_resid_blocks(n3), &p));
    red.partials = static_cast<double *>(p);
    const double2 *b = static_cast<const double2 *>(b_dev);
    double2 *x = static_cast<double2 *>(x_dev);
    // r = b - A x, d = N(r), r' = r - A d
    HISQ_TRY(apply_mdagm(g, two_m, x, t, nrhs, s));
    HISQ_TRY(mixed_resid(b, t, r, n3, nrhs, nullptr, r2, red, s));
    HISQ_TRY(apply_net(n, reinterpret_cast<const dvec2 *>(r), reinterpret_cast<dvec2 *>(d), nrhs,
                       flags, s));
    HISQ_TRY(apply_mdagm(g, two_m, d, t, nrhs, s));
    if (n_ev > 0) {
        // Galerkin correction on the deflation space: d += V L^-1 V^H (r - A d).
        // With x deflated, V^H r = 0 and this removes V V^H d: the network
        // must not put error back into the lowest modes, where CG is slowest.
        void *q = nullptr;
        HISQ_TRY(ws_get(n, "guess_c", vb, &q));
        double2 *c = static_cast<double2 *>(q);
        HISQ_TRY(mixed_resid(r, t, t, n3, nrhs, nullptr, r2 + nrhs, red, s));
        HISQ_TRY(hisq_deflate(g, n_ev, evecs_dev, evec_prec, evals_host, two_m, t, c, nrhs, s));
        hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n3 * nrhs, 4096)), dim3(kBS), 0, s,
                           reinterpret_cast<dvec2 *>(d), reinterpret_cast<const dvec2 *>(c),
                           n3 * nrhs);
        HISQ_HIP(hipGetLastError());
        HISQ_TRY(apply_mdagm(g, two_m, d, t, nrhs, s));
    }
    HISQ_TRY(mixed_resid(r, t, t, n3, nrhs, nullptr, r2 + nrhs, red, s));
    hipLaunchKernelGGL(k_keep_add, dim3(blocks_for(n3, 2048), nrhs), dim3(kBS), 0, s,
                       reinterpret_cast<dvec2 *>(x), reinterpret_cast<const dvec2 *>(d), r2, r2 + nrhs,
                       keep, n3);
    HISQ_HIP(hipGetLastError());
    if (kept_host) {
        HISQ_HIP(hipMemcpyAsync(kept_host, keep, sizeof(int) * nrhs, hipMemcpyDeviceToHost, s));
        HISQ_HIP(hipStreamSynchronize(s));
    }
    return HISQ_OK;
}

}  // extern "C"
