// BF16 storage for the half stencil: links and vectors held as bfloat16 pairs
// (8 significant bits), arithmetic in FP32.  Section 3 of arXiv:2502.00152
// describes the production solve as mixed-precision CG in which the bulk of
// the operator runs in reduced precision and the reliable updates restore
// FP64 accuracy; bfloat16 halves the bytes of FP32 storage again.  Two
// variants: BF16 vectors with BF16 links (the operators at HISQ_BF16), and FP32
// vectors with BF16 links (the sloppy operator of the CG at sloppy_prec =
// HISQ_BF16: the iterated vectors keep FP32, the links - two thirds of the
// bytes of a 12-RHS launch and 96% of a 1-RHS one - are read at half size).
// BF16 links are made once per gauge handle from the FP64 ones.
#include "dslash_kernel.h"

namespace hisq {

hisq_status dslash_check_shape(const DslashShape &sh);

namespace {

constexpr int kBS = 256;

// FP64 -> bfloat16, rounded to nearest even in one step: round to FP32 toward
// zero, mark inexactness in the last FP32 bit (round to odd), then round that
// to bfloat16 to nearest even (FP32 keeps 16 bits more than bfloat16, so the
// two steps give the directly rounded result).
__device__ __forceinline__ uint32_t bf16_of_double(double d) {
    float f = __double2float_rz(d);
    uint32_t u = __float_as_uint(f);
    if ((double)f != d) u |= 1u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

__global__ __launch_bounds__(kBS) void k_links_to_bf16(const double2 *__restrict__ src,
                                                       bf16c *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const double2 v = src[i];
        dst[i] = bf16_of_double(v.x) | (bf16_of_double(v.y) << 16);
    }
}

}  // namespace

hisq_status ensure_links_bf16(hisq_gauge_s *g, hipStream_t s) {
    if (g->fat16[0]) return HISQ_OK;
    const int64_t n = link_array_entries(g->geom.vh);
    for (int p = 0; p < 2; ++p) {
        if (hipMalloc(&g->fat16[p], sizeof(bf16c) * n) != hipSuccess ||
            hipMalloc(&g->lng16[p], sizeof(bf16c) * n) != hipSuccess)
            return fail(HISQ_ERR_OOM, "device allocation of the BF16 links");
    }
    const int nb = (int)std::min<int64_t>((n + kBS - 1) / kBS, 8192);
    for (int p = 0; p < 2; ++p) {
        hipLaunchKernelGGL(k_links_to_bf16, dim3(nb), dim3(kBS), 0, s, g->fat[p], g->fat16[p], n);
        hipLaunchKernelGGL(k_links_to_bf16, dim3(nb), dim3(kBS), 0, s, g->lng[p], g->lng16[p], n);
    }
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status convert_double_to_bf16(const double2 *src, bf16c *dst, int64_t n, hipStream_t s) {
    if (n == 0) return HISQ_OK;
    const int nb = (int)std::min<int64_t>((n + kBS - 1) / kBS, 16384);
    hipLaunchKernelGGL(k_links_to_bf16, dim3(nb), dim3(kBS), 0, s, src, dst, n);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status launch_dslash_bf16(hisq_gauge_s *g, int out_parity, const bf16c *in, bf16c *out,
                               int nrhs, const bf16c *aux, double ca, const bf16c *aux2,
                               double cb, double cd, hipStream_t s) {
    HISQ_TRY(ensure_links_bf16(g, s));
    const bf16c *fat[2] = {g->fat16[0], g->fat16[1]};
    const bf16c *lng[2] = {g->lng16[0], g->lng16[1]};
    const DslashShape sh = dslash_pick_shape(nrhs, g->geom.vh, 2, false, g->geom);
    HISQ_TRY(dslash_check_shape(sh));
    ProfileScope prof(aux2 ? "dslash_bf16_aux2" : aux ? "dslash_bf16_aux" : "dslash_bf16", s);
    return dslash_impl::launch_dslash_t<float, bf16c, bf16c>(g->geom, fat, lng, out_parity, in, out,
                                                             nrhs, aux, ca, aux2, cb, cd, nullptr,
                                                             sh, s);
}

hisq_status launch_dslash_f32_bl(hisq_gauge_s *g, int out_parity, const float2 *in, float2 *out,
                                 int nrhs, const float2 *aux, double ca, double cd,
                                 double *partials, hipStream_t s, const double *ca_rhs,
                                 const int *rhs_status) {
    HISQ_TRY(ensure_links_bf16(g, s));
    using V = vec2<float>;
    const bf16c *fat[2] = {g->fat16[0], g->fat16[1]};
    const bf16c *lng[2] = {g->lng16[0], g->lng16[1]};
    const DslashShape sh = dslash_pick_shape(nrhs, g->geom.vh, 4, false, g->geom);
    HISQ_TRY(dslash_check_shape(sh));
    ProfileScope prof(aux ? "dslash_f32bl_aux" : "dslash_f32bl", s);
    return dslash_impl::launch_dslash_t<float, V, bf16c>(
        g->geom, fat, lng, out_parity, reinterpret_cast<const V *>(in), reinterpret_cast<V *>(out),
        nrhs, reinterpret_cast<const V *>(aux), ca, nullptr, 0.0, cd, partials, sh, s, ca_rhs,
        rhs_status);
}

hisq_status apply_mdagm_bf16(hisq_gauge_s *g, double two_m, const bf16c *in, bf16c *out, int nrhs,
                             hipStream_t s) {
    void *tmp = nullptr;
    HISQ_TRY(g->ws.get("mdagm_tmp16", sizeof(bf16c) * 3 * (size_t)g->geom.vh * nrhs, &tmp));
    bf16c *t = static_cast<bf16c *>(tmp);
    HISQ_TRY(launch_dslash_bf16(g, 1, in, t, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, s));
    return launch_dslash_bf16(g, 0, t, out, nrhs, in, two_m * two_m, nullptr, 0.0, -1.0, s);
}

}  // namespace hisq
