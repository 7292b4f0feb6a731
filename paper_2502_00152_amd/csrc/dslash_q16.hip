// 16-bit fixed-point links for the sloppy operator of the mixed-precision CG
// (arXiv:2502.00152, section 2: the conventional solve is mixed-precision CG;
// the reliable updates it cites were introduced with such a half-precision
// format).  Every link component is stored as round(x / step), step = (largest
// |component| over fat and long links of the handle) / 32767, an absolute
// error <= step / 2 per component; vectors stay FP32 and the arithmetic is
// FP32.  The kernel multiplies the integers as floats and the launcher folds
// step into the stencil coefficient cd.  Half the link bytes of FP32, about
// 4e-5 relative accuracy for unitary links (BF16: 2e-3).  The stencil on
// 16-bit vectors reads a second copy whose step is chosen per field so that
// the integer products of a link row and a colour vector sum exactly in int32
// (largest / ~26700 for near-unitary links, never coarser than / 10922).
#include <algorithm>
#include <cmath>
#include <vector>

#include "dslash_kernel.h"

namespace hisq {

hisq_status dslash_check_shape(const DslashShape &sh);

namespace {

constexpr int kBS = 256;
constexpr int kMaxBlocks = 1024;

// per-block max |component| (re and im) of n complex numbers
__global__ __launch_bounds__(kBS) void k_absmax(const double2 *__restrict__ src, int64_t n,
                                                double *__restrict__ partials) {
    __shared__ double m[kBS];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const double2 a = src[i];
        v = fmax(v, fmax(fabs(a.x), fabs(a.y)));
    }
    m[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBS / 2; w > 0; w /= 2) {
        if ((int)threadIdx.x < w) m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = m[0];
}

// per-block max over link rows of sum_b (|Re U_ab| + |Im U_ab|), for nslots
// site slots of the tiled layout [tile][9 entries][kLinkTile sites]
__global__ __launch_bounds__(kBS) void k_rowl1max(const double2 *__restrict__ src, int64_t nslots,
                                                  double *__restrict__ partials) {
    __shared__ double m[kBS];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < nslots;
         i += (int64_t)gridDim.x * kBS) {
        const int64_t base = (i / kLinkTile) * 9 * kLinkTile + (i % kLinkTile);
        for (int a = 0; a < 3; ++a) {
            double r = 0.0;
            for (int b = 0; b < 3; ++b) {
                const double2 u = src[base + (3 * a + b) * kLinkTile];
                r += fabs(u.x) + fabs(u.y);
            }
            v = fmax(v, r);
        }
    }
    m[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBS / 2; w > 0; w /= 2) {
        if ((int)threadIdx.x < w) m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = m[0];
}

__device__ __forceinline__ uint32_t q16_of(double x, double inv_step, int qmax) {
    const long long q = llrint(x * inv_step);
    const int c = (int)(q > qmax ? qmax : (q < -qmax ? -qmax : q));
    return (uint32_t)c & 0xffffu;
}

// Entry i of the tiled layout [4 mu][tile][9 k][kLinkTile] rounded to 16
// bits; split: stored at its place in the q16s layout instead (per direction
// entries 0-3 of each site, then 4-7, then 8; vhp = tiles * kLinkTile sites).
__global__ __launch_bounds__(kBS) void k_links_to_q16(const double2 *__restrict__ src,
                                                      q16c *__restrict__ dst, int64_t n,
                                                      double inv_step, int qmax, bool split,
                                                      int64_t tiles) {
    const int64_t vhp = tiles * kLinkTile;
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const double2 v = src[i];
        int64_t o = i;
        if (split) {
            const int64_t lane = i % kLinkTile, r = i / kLinkTile;
            const int k = (int)(r % 9);
            const int64_t rt = r / 9, tile = rt % tiles, mu = rt / tiles;
            const int64_t cb = tile * kLinkTile + lane;
            const int part = k < 4 ? 0 : (k < 8 ? 1 : 2);
            o = mu * 9 * vhp + part * 4 * vhp + (part < 2 ? cb * 4 + (k - 4 * part) : cb);
        }
        dst[o] = (q16c)(q16_of(v.x, inv_step, qmax) | (q16_of(v.y, inv_step, qmax) << 16));
    }
}

// largest |component| over the fat and long links (once per handle)
hisq_status link_absmax(hisq_gauge_s *g, hipStream_t s, double *mx_out) {
    if (g->link_absmax >= 0.0) {
        *mx_out = g->link_absmax;
        return HISQ_OK;
    }
    const int64_t n = link_array_entries(g->geom.vh);
    const int nb = (int)std::min<int64_t>((n + kBS - 1) / kBS, kMaxBlocks);
    void *p = nullptr;
    HISQ_TRY(g->ws.get("q16_absmax", sizeof(double) * 4 * kMaxBlocks, &p));
    double *part = static_cast<double *>(p);
    const double2 *arrays[4] = {g->fat[0], g->fat[1], g->lng[0], g->lng[1]};
    for (int a = 0; a < 4; ++a)
        hipLaunchKernelGGL(k_absmax, dim3(nb), dim3(kBS), 0, s, arrays[a], n, part + a * kMaxBlocks);
    HISQ_HIP(hipGetLastError());
    std::vector<double> h(4 * (size_t)kMaxBlocks);
    HISQ_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    double mx = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < nb; ++b) mx = std::max(mx, h[(size_t)a * kMaxBlocks + b]);
    g->link_absmax = mx;
    *mx_out = mx;
    return HISQ_OK;
}

// largest row sum of |Re| + |Im| over the fat and long links
hisq_status link_rowl1max(hisq_gauge_s *g, hipStream_t s, double *out) {
    const int64_t nslots = link_array_entries(g->geom.vh) / 9;
    const int nb = (int)std::min<int64_t>((nslots + kBS - 1) / kBS, kMaxBlocks);
    void *p = nullptr;
    HISQ_TRY(g->ws.get("q16_absmax", sizeof(double) * 4 * kMaxBlocks, &p));
    double *part = static_cast<double *>(p);
    const double2 *arrays[4] = {g->fat[0], g->fat[1], g->lng[0], g->lng[1]};
    for (int a = 0; a < 4; ++a)
        hipLaunchKernelGGL(k_rowl1max, dim3(nb), dim3(kBS), 0, s, arrays[a], nslots,
                           part + a * kMaxBlocks);
    HISQ_HIP(hipGetLastError());
    std::vector<double> h(4 * (size_t)kMaxBlocks);
    HISQ_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    double mx = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < nb; ++b) mx = std::max(mx, h[(size_t)a * kMaxBlocks + b]);
    *out = mx;
    return HISQ_OK;
}

// fixed-point copies of both link fields, components in [-qmax, qmax], in
// the tiled layout or (split) the q16s layout
hisq_status make_q16_links(hisq_gauge_s *g, int qmax, bool split, int32_t *(&fat)[2],
                           int32_t *(&lng)[2], double *step_out, hipStream_t s) {
    double mx = 0.0;
    HISQ_TRY(link_absmax(g, s, &mx));
    const int64_t n = link_array_entries(g->geom.vh);
    const double step = mx > 0.0 ? mx / qmax : 1.0;
    for (int q = 0; q < 2; ++q) {
        if (hipMalloc(&fat[q], sizeof(q16c) * n) != hipSuccess ||
            hipMalloc(&lng[q], sizeof(q16c) * n) != hipSuccess)
            return fail(HISQ_ERR_OOM, "device allocation of the 16-bit links");
    }
    const int nc = (int)std::min<int64_t>((n + kBS - 1) / kBS, 8192);
    for (int q = 0; q < 2; ++q) {
        hipLaunchKernelGGL(k_links_to_q16, dim3(nc), dim3(kBS), 0, s, g->fat[q], fat[q], n,
                           1.0 / step, qmax, split, link_tiles(g->geom.vh));
        hipLaunchKernelGGL(k_links_to_q16, dim3(nc), dim3(kBS), 0, s, g->lng[q], lng[q], n,
                           1.0 / step, qmax, split, link_tiles(g->geom.vh));
    }
    HISQ_HIP(hipGetLastError());
    *step_out = step;
    return HISQ_OK;
}

}  // namespace

hisq_status ensure_links_q16(hisq_gauge_s *g, hipStream_t s) {
    if (g->fatq[0]) return HISQ_OK;
    return make_q16_links(g, 32767, false, g->fatq, g->lngq, &g->q16_step, s);
}

// The copy read by the stencil on 16-bit vectors, whose integer dot products
// must not overflow for any vector with components up to 32767: Re and Im of
// a row times a vector are bounded by 32767 times the row's integer L1 norm
// (sum of |Re| + |Im|), which is at most rowl1 * qmax / absmax + 3 after
// rounding; qmax <= 65535 absmax / rowl1 keeps that below 65538, and
// 65538 * 32767 < 2^31.  Near-unitary links (row L1 <= sqrt 6 absmax) give
// qmax ~ 26700; kQLinkNarrow covers any field.
int q16n_qmax(double absmax, double rowl1) {
    if (!(absmax > 0.0) || !(rowl1 > 0.0)) return kQLinkNarrow;
    const double q = std::floor(65535.0 * absmax / rowl1) - 1.0;
    return (int)std::max<double>(kQLinkNarrow, std::min<double>(32767.0, q));
}

hisq_status ensure_links_q16n(hisq_gauge_s *g, hipStream_t s) {
    if (g->fatn[0]) return HISQ_OK;
    double mx = 0.0, rl1 = 0.0;
    HISQ_TRY(link_absmax(g, s, &mx));
    HISQ_TRY(link_rowl1max(g, s, &rl1));
    g->qn_max = q16n_qmax(mx, rl1);
    return make_q16_links(g, g->qn_max, true, g->fatn, g->lngn, &g->qn_step, s);
}

hisq_status launch_dslash_f32_q16(hisq_gauge_s *g, int out_parity, const float2 *in, float2 *out,
                                  int nrhs, const float2 *aux, double ca, double cd,
                                  double *partials, hipStream_t s, const double *ca_rhs,
                                  const int *rhs_status) {
    HISQ_TRY(ensure_links_q16(g, s));
    using V = vec2<float>;
    const q16c *fat[2] = {g->fatq[0], g->fatq[1]};
    const q16c *lng[2] = {g->lngq[0], g->lngq[1]};
    const DslashShape sh = dslash_pick_shape(nrhs, g->geom.vh, 4, true, g->geom);
    HISQ_TRY(dslash_check_shape(sh));
    ProfileScope prof(aux ? "dslash_q16_aux" : "dslash_q16", s);
    return dslash_impl::launch_dslash_t<float, V, q16c>(
        g->geom, fat, lng, out_parity, reinterpret_cast<const V *>(in), reinterpret_cast<V *>(out),
        nrhs, reinterpret_cast<const V *>(aux), ca, nullptr, 0.0, cd * g->q16_step, partials, sh, s,
        ca_rhs, rhs_status);
}

hisq_status apply_mdagm_q16(hisq_gauge_s *g, double two_m, const float2 *in, float2 *out, int nrhs,
                            hipStream_t s) {
    void *tmp = nullptr;
    HISQ_TRY(g->ws.get("mdagm_tmp32", sizeof(float2) * 3 * (size_t)g->geom.vh * nrhs, &tmp));
    float2 *t = static_cast<float2 *>(tmp);
    HISQ_TRY(launch_dslash_f32_q16(g, 1, in, t, nrhs, nullptr, 0.0, 1.0, nullptr, s));
    return launch_dslash_f32_q16(g, 0, t, out, nrhs, in, two_m * two_m, -1.0, nullptr, s);
}

}  // namespace hisq

namespace hisq {

// 16-bit vectors (packed h16p fields) and 16-bit links (q16s layout): the
// sloppy operator at sloppy_prec = HISQ_HALF.  The kernel sums the integer
// products of a link row and a colour vector exactly in 32 bits and scales by
// the neighbour's norm; the link step and 1/32767 of the vectors fold into cd.
hisq_status launch_dslash_h16(hisq_gauge_s *g, int out_parity, const void *in, void *out,
                              int nrhs, const void *aux, double ca, double cd, double *partials,
                              hipStream_t s, const double *ca_rhs, const int *rhs_status) {
    HISQ_TRY(ensure_links_q16n(g, s));
    const q16s *fat[2] = {reinterpret_cast<const q16s *>(g->fatn[0]),
                          reinterpret_cast<const q16s *>(g->fatn[1])};
    const q16s *lng[2] = {reinterpret_cast<const q16s *>(g->lngn[0]),
                          reinterpret_cast<const q16s *>(g->lngn[1])};
    const DslashShape sh = dslash_pick_shape(nrhs, g->geom.vh, 2, true, g->geom, aux == nullptr);
    HISQ_TRY(dslash_check_shape(sh));
    ProfileScope prof(aux ? "dslash_h16_aux" : "dslash_h16", s);
    return dslash_impl::launch_dslash_t<float, h16p, q16s>(
        g->geom, fat, lng, out_parity, static_cast<const h16p *>(in), static_cast<h16p *>(out),
        nrhs, static_cast<const h16p *>(aux), ca, nullptr, 0.0, cd * g->qn_step / kQ16, partials,
        sh, s, ca_rhs, rhs_status);
}

}  // namespace hisq
