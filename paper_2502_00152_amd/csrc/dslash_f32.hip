// FP32 half stencil and M^H M: the sloppy operator of the mixed-precision CG
// (arXiv:2502.00152, section 2: the conventional solve is mixed-precision CG;
// links and vectors stored in FP32, arithmetic in FP32, the CG's dot products
// accumulated in FP64).  FP32 links are made once per gauge handle from the
// FP64 ones.
#include "dslash_kernel.h"

namespace hisq {

hisq_status dslash_check_shape(const DslashShape &sh);

namespace {

constexpr int kBS = 256;

__global__ __launch_bounds__(kBS) void k_links_to_f32(const double2 *__restrict__ src,
                                                      float2 *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const double2 v = src[i];
        dst[i] = make_float2((float)v.x, (float)v.y);
    }
}

}  // namespace

hisq_status ensure_links_f32(hisq_gauge_s *g, hipStream_t s) {
    if (g->fat32[0]) return HISQ_OK;
    const int64_t n = link_array_entries(g->geom.vh);
    for (int p = 0; p < 2; ++p) {
        if (hipMalloc(&g->fat32[p], sizeof(float2) * n) != hipSuccess ||
            hipMalloc(&g->lng32[p], sizeof(float2) * n) != hipSuccess)
            return fail(HISQ_ERR_OOM, "device allocation of the FP32 links");
    }
    const int nb = (int)std::min<int64_t>((n + kBS - 1) / kBS, 8192);
    for (int p = 0; p < 2; ++p) {
        hipLaunchKernelGGL(k_links_to_f32, dim3(nb), dim3(kBS), 0, s, g->fat[p], g->fat32[p], n);
        hipLaunchKernelGGL(k_links_to_f32, dim3(nb), dim3(kBS), 0, s, g->lng[p], g->lng32[p], n);
    }
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status launch_dslash_f32(hisq_gauge_s *g, int out_parity, const float2 *in, float2 *out,
                              int nrhs, const float2 *aux, double ca, const float2 *aux2, double cb,
                              double cd, double *partials, hipStream_t s, const double *ca_rhs,
                              const int *rhs_status) {
    HISQ_TRY(ensure_links_f32(g, s));
    using V = vec2<float>;
    const V *fat[2] = {reinterpret_cast<const V *>(g->fat32[0]),
                       reinterpret_cast<const V *>(g->fat32[1])};
    const V *lng[2] = {reinterpret_cast<const V *>(g->lng32[0]),
                       reinterpret_cast<const V *>(g->lng32[1])};
    const DslashShape sh = dslash_pick_shape(nrhs, g->geom.vh, sizeof(float), false, g->geom);
    HISQ_TRY(dslash_check_shape(sh));
    ProfileScope prof(aux2 ? "dslash_f32_aux2" : aux ? "dslash_f32_aux" : "dslash_f32", s);
    return dslash_impl::launch_dslash_t<float>(
        g->geom, fat, lng, out_parity, reinterpret_cast<const V *>(in), reinterpret_cast<V *>(out),
        nrhs, reinterpret_cast<const V *>(aux), ca, reinterpret_cast<const V *>(aux2), cb, cd,
        partials, sh, s, ca_rhs, rhs_status);
}

hisq_status apply_mdagm_f32(hisq_gauge_s *g, double two_m, const float2 *in, float2 *out, int nrhs,
                            double *partials, hipStream_t s) {
    void *tmp = nullptr;
    HISQ_TRY(g->ws.get("mdagm_tmp32", sizeof(float2) * 3 * (size_t)g->geom.vh * nrhs, &tmp));
    float2 *t = static_cast<float2 *>(tmp);
    HISQ_TRY(launch_dslash_f32(g, 1, in, t, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, nullptr, s));
    HISQ_TRY(launch_dslash_f32(g, 0, t, out, nrhs, in, two_m * two_m, nullptr, 0.0, -1.0, partials,
                               s));
    return HISQ_OK;
}

}  // namespace hisq
