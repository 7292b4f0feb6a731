// extern "C" entry points: gauge handles, layout conversion and the
// stencil-based operators.  The CG, deflation and eigensolver entry points
// live in cg.hip, deflate.hip and eigensolve.hip.
#include <cmath>
#include <new>

#include "hisq_internal.h"

using namespace hisq;

namespace hisq {

hisq_status check_gauge(hisq_gauge g) {
    if (!g) return fail(HISQ_ERR_INVALID_ARG, "null gauge handle");
    HISQ_HIP(hipSetDevice(g->device));
    return HISQ_OK;
}

hisq_status check_vec(const void *p, const char *name) {
    if (!p) return fail(HISQ_ERR_INVALID_ARG, std::string(name) + " is null");
    if (reinterpret_cast<uintptr_t>(p) % 16)
        return fail(HISQ_ERR_INVALID_ARG, std::string(name) + " is not 16-byte aligned");
    return HISQ_OK;
}

hisq_status check_nrhs(int nrhs) {
    if (nrhs < 1 || nrhs > 4096) return fail(HISQ_ERR_INVALID_ARG, "nrhs out of range");
    return HISQ_OK;
}

hisq_status check_prec(hisq_prec p) {
    if (p == HISQ_FP64 || p == HISQ_FP32 || p == HISQ_BF16 || p == HISQ_Q16 || p == HISQ_HALF)
        return HISQ_OK;
    return fail(HISQ_ERR_INVALID_ARG, "unknown precision");
}

hisq_status check_mass(double two_m, bool positive) {
    if (!std::isfinite(two_m) || two_m < 0.0 || (positive && two_m == 0.0))
        return fail(HISQ_ERR_INVALID_ARG, positive ? "two_m must be finite and > 0"
                                                   : "two_m must be finite and >= 0");
    return HISQ_OK;
}

}  // namespace hisq

extern "C" {

hisq_status hisq_gauge_create(hisq_gauge *out, const int dims[4], const void *fat_dev,
                              const void *long_dev, double c_fat, double c_long,
                              unsigned flags, void *stream) {
    if (!out || !dims) return fail(HISQ_ERR_INVALID_ARG, "hisq_gauge_create: null argument");
    *out = nullptr;
    int64_t V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 2 || dims[mu] % 2)
            return fail(HISQ_ERR_INVALID_ARG, "every lattice extent must be even and >= 2");
        V *= dims[mu];
    }
    if (V >= (int64_t(1) << 31))
        return fail(HISQ_ERR_INVALID_ARG, "lattice volume must be below 2^31 sites");
    HISQ_TRY(check_vec(fat_dev, "fat_dev"));
    HISQ_TRY(check_vec(long_dev, "long_dev"));
    if (!std::isfinite(c_fat) || !std::isfinite(c_long))
        return fail(HISQ_ERR_INVALID_ARG, "link coefficients must be finite");
    if (flags & ~(unsigned)(HISQ_GAUGE_FOLD_PHASES | HISQ_GAUGE_ANTIPERIODIC_T))
        return fail(HISQ_ERR_INVALID_ARG, "unknown gauge flags");

    hisq_gauge g = new (std::nothrow) hisq_gauge_s();
    if (!g) return fail(HISQ_ERR_OOM, "host allocation of the gauge handle");
    g->geom.X = dims[0];
    g->geom.Y = dims[1];
    g->geom.Z = dims[2];
    g->geom.T = dims[3];
    g->geom.Xh = dims[0] / 2;
    g->geom.vh = (int)(V / 2);
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return fail(HISQ_ERR_HIP, "hipGetDevice failed");
    }
    const size_t per = sizeof(double2) * (size_t)link_array_entries(g->geom.vh);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int p = 0; p < 2; ++p) {
        if (hipMalloc(&g->fat[p], per) != hipSuccess || hipMalloc(&g->lng[p], per) != hipSuccess) {
            hisq_gauge_destroy(g);
            return fail(HISQ_ERR_OOM, "device allocation of the links");
        }
        // the padding of the last tile is never read; keep it defined
        if (hipMemsetAsync(g->fat[p], 0, per, s) != hipSuccess ||
            hipMemsetAsync(g->lng[p], 0, per, s) != hipSuccess) {
            hisq_gauge_destroy(g);
            return fail(HISQ_ERR_HIP, "clearing the link arrays");
        }
    }
    hisq_status st = launch_pack_links(g, static_cast<const double2 *>(fat_dev), g->fat, c_fat,
                                       flags, false, s);
    if (st == HISQ_OK)
        st = launch_pack_links(g, static_cast<const double2 *>(long_dev), g->lng, c_long, flags,
                               true, s);
    if (st == HISQ_OK && hipStreamSynchronize(s) != hipSuccess)
        st = fail(HISQ_ERR_HIP, "link packing failed");
    if (st != HISQ_OK) {
        std::string msg = hisq_last_error();
        hisq_gauge_destroy(g);
        return fail(st, msg);
    }
    *out = g;
    return HISQ_OK;
}

hisq_status hisq_gauge_destroy(hisq_gauge g) {
    if (!g) return HISQ_OK;
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    for (int p = 0; p < 2; ++p) {
        if (g->fat[p]) (void)hipFree(g->fat[p]);
        if (g->lng[p]) (void)hipFree(g->lng[p]);
        if (g->fat32[p]) (void)hipFree(g->fat32[p]);
        if (g->lng32[p]) (void)hipFree(g->lng32[p]);
        if (g->fat16[p]) (void)hipFree(g->fat16[p]);
        if (g->lng16[p]) (void)hipFree(g->lng16[p]);
        if (g->fatq[p]) (void)hipFree(g->fatq[p]);
        if (g->lngq[p]) (void)hipFree(g->lngq[p]);
        if (g->fatn[p]) (void)hipFree(g->fatn[p]);
        if (g->lngn[p]) (void)hipFree(g->lngn[p]);
    }
    g->ws.release();
    if (g->cg_stream) (void)hipStreamDestroy(g->cg_stream);
    delete g;
    return HISQ_OK;
}

int64_t hisq_gauge_half_volume(hisq_gauge g) { return g ? g->geom.vh : 0; }

hisq_status hisq_spinor_split(hisq_gauge g, const void *full_dev, void *even_dev,
                              void *odd_dev, int nrhs, void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_vec(full_dev, "full_dev"));
    if (even_dev) HISQ_TRY(check_vec(even_dev, "even_dev"));
    if (odd_dev) HISQ_TRY(check_vec(odd_dev, "odd_dev"));
    return launch_split(g, static_cast<const double2 *>(full_dev),
                        static_cast<double2 *>(even_dev), static_cast<double2 *>(odd_dev), nrhs,
                        static_cast<hipStream_t>(stream));
}

hisq_status hisq_spinor_merge(hisq_gauge g, const void *even_dev, const void *odd_dev,
                              void *full_dev, int nrhs, void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_vec(full_dev, "full_dev"));
    if (even_dev) HISQ_TRY(check_vec(even_dev, "even_dev"));
    if (odd_dev) HISQ_TRY(check_vec(odd_dev, "odd_dev"));
    return launch_merge(g, static_cast<const double2 *>(even_dev),
                        static_cast<const double2 *>(odd_dev), static_cast<double2 *>(full_dev),
                        nrhs, static_cast<hipStream_t>(stream));
}

hisq_status hisq_convert_vectors(const void *src_dev, hisq_prec src_prec, void *dst_dev,
                                 hisq_prec dst_prec, int64_t n_complex, void *stream) {
    HISQ_TRY(check_vec(src_dev, "src_dev"));
    HISQ_TRY(check_vec(dst_dev, "dst_dev"));
    if (n_complex < 0) return fail(HISQ_ERR_INVALID_ARG, "n_complex must be >= 0");
    auto bytes = [](hisq_prec p) -> size_t {
        return p == HISQ_FP64 ? sizeof(double2)
             : p == HISQ_FP32 ? sizeof(float2)
             : p == HISQ_BF16 ? sizeof(uint32_t) : 0;
    };
    const size_t sb = bytes(src_prec), db = bytes(dst_prec);
    if (!sb || !db)
        return fail(HISQ_ERR_INVALID_ARG, "precision must be HISQ_FP64, HISQ_FP32 or HISQ_BF16");
    const char *s0 = static_cast<const char *>(src_dev);
    const char *d0 = static_cast<const char *>(dst_dev);
    if (n_complex > 0 && s0 < d0 + db * n_complex && d0 < s0 + sb * n_complex)
        return fail(HISQ_ERR_INVALID_ARG, "src and dst must not overlap");
    return convert_vectors(src_dev, src_prec, dst_dev, dst_prec, n_complex,
                           static_cast<hipStream_t>(stream));
}

hisq_status hisq_dslash_eo(hisq_gauge g, int out_parity, const void *in_dev, void *out_dev,
                           int nrhs, hisq_prec prec, void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_prec(prec));
    if (out_parity != 0 && out_parity != 1)
        return fail(HISQ_ERR_INVALID_ARG, "out_parity must be 0 (even) or 1 (odd)");
    HISQ_TRY(check_vec(in_dev, "in_dev"));
    HISQ_TRY(check_vec(out_dev, "out_dev"));
    if (in_dev == out_dev) return fail(HISQ_ERR_INVALID_ARG, "in and out must not overlap");
    if (prec == HISQ_FP32)
        return launch_dslash_f32(g, out_parity, static_cast<const float2 *>(in_dev),
                                 static_cast<float2 *>(out_dev), nrhs, nullptr, 0.0, nullptr, 0.0,
                                 1.0, nullptr, static_cast<hipStream_t>(stream));
    if (prec == HISQ_HALF)
        return apply_dslash_half(g, out_parity, static_cast<const float2 *>(in_dev),
                                 static_cast<float2 *>(out_dev), nrhs,
                                 static_cast<hipStream_t>(stream));
    if (prec == HISQ_Q16)
        return launch_dslash_f32_q16(g, out_parity, static_cast<const float2 *>(in_dev),
                                     static_cast<float2 *>(out_dev), nrhs, nullptr, 0.0, 1.0,
                                     nullptr, static_cast<hipStream_t>(stream));
    if (prec == HISQ_BF16)
        return launch_dslash_bf16(g, out_parity, static_cast<const uint32_t *>(in_dev),
                                  static_cast<uint32_t *>(out_dev), nrhs, nullptr, 0.0, nullptr,
                                  0.0, 1.0, static_cast<hipStream_t>(stream));
    return launch_dslash(g, out_parity, static_cast<const double2 *>(in_dev),
                         static_cast<double2 *>(out_dev), nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE,
                         nullptr, nullptr, static_cast<hipStream_t>(stream));
}

hisq_status hisq_mdagm(hisq_gauge g, double two_m, const void *in_e_dev, void *out_e_dev,
                       int nrhs, hisq_prec prec, void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_prec(prec));
    HISQ_TRY(check_mass(two_m, false));
    HISQ_TRY(check_vec(in_e_dev, "in_e_dev"));
    HISQ_TRY(check_vec(out_e_dev, "out_e_dev"));
    if (in_e_dev == out_e_dev) return fail(HISQ_ERR_INVALID_ARG, "in and out must not overlap");
    if (prec == HISQ_FP32)
        return apply_mdagm_f32(g, two_m, static_cast<const float2 *>(in_e_dev),
                               static_cast<float2 *>(out_e_dev), nrhs, nullptr,
                               static_cast<hipStream_t>(stream));
    if (prec == HISQ_HALF)
        return apply_mdagm_half(g, two_m, static_cast<const float2 *>(in_e_dev),
                                static_cast<float2 *>(out_e_dev), nrhs,
                                static_cast<hipStream_t>(stream));
    if (prec == HISQ_Q16)
        return apply_mdagm_q16(g, two_m, static_cast<const float2 *>(in_e_dev),
                               static_cast<float2 *>(out_e_dev), nrhs,
                               static_cast<hipStream_t>(stream));
    if (prec == HISQ_BF16)
        return apply_mdagm_bf16(g, two_m, static_cast<const uint32_t *>(in_e_dev),
                                static_cast<uint32_t *>(out_e_dev), nrhs,
                                static_cast<hipStream_t>(stream));
    return apply_mdagm(g, two_m, static_cast<const double2 *>(in_e_dev),
                       static_cast<double2 *>(out_e_dev), nrhs, static_cast<hipStream_t>(stream));
}

hisq_status hisq_prepare_source(hisq_gauge g, double two_m, const void *eta_e_dev,
                                const void *eta_o_dev, void *y_e_dev, int nrhs, void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_mass(two_m, false));
    HISQ_TRY(check_vec(eta_e_dev, "eta_e_dev"));
    HISQ_TRY(check_vec(eta_o_dev, "eta_o_dev"));
    HISQ_TRY(check_vec(y_e_dev, "y_e_dev"));
    if (y_e_dev == eta_o_dev) return fail(HISQ_ERR_INVALID_ARG, "y_e must not overlap eta_o");
    // y_e = 2m eta_e - D_eo eta_o
    return launch_dslash(g, 0, static_cast<const double2 *>(eta_o_dev),
                         static_cast<double2 *>(y_e_dev), nrhs,
                         static_cast<const double2 *>(eta_e_dev), two_m, nullptr, 0.0, -1.0, FIN_NONE, nullptr,
                         nullptr, static_cast<hipStream_t>(stream));
}

hisq_status hisq_reconstruct_odd(hisq_gauge g, double two_m, const void *psi_e_dev,
                                 const void *eta_o_dev, void *psi_o_dev, int nrhs,
                                 void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_mass(two_m, true));
    HISQ_TRY(check_vec(psi_e_dev, "psi_e_dev"));
    HISQ_TRY(check_vec(eta_o_dev, "eta_o_dev"));
    HISQ_TRY(check_vec(psi_o_dev, "psi_o_dev"));
    if (psi_o_dev == psi_e_dev) return fail(HISQ_ERR_INVALID_ARG, "psi_o must not overlap psi_e");
    // psi_o = (eta_o - D_oe psi_e) / (2m)
    const double inv = 1.0 / two_m;
    return launch_dslash(g, 1, static_cast<const double2 *>(psi_e_dev),
                         static_cast<double2 *>(psi_o_dev), nrhs,
                         static_cast<const double2 *>(eta_o_dev), inv, nullptr, 0.0, -inv, FIN_NONE, nullptr,
                         nullptr, static_cast<hipStream_t>(stream));
}

}  // extern "C"
