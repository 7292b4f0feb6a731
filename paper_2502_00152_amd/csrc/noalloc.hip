// hisq_mdagm_noalloc: the even-site normal operator (2m)^2 - D_eo D_oe of
// hisq_mdagm (arXiv:2502.00152, section 2: the even-odd preconditioned
// operator of Eq. (1)) for callers that cannot allocate device memory.  The
// odd-parity temporary between the two half stencils is a file-scope device
// array instead of the handle's grown-on-demand scratch; the kernels are the
// ones hisq_mdagm launches, with the same launch shapes.
#include <mutex>

#include "hisq_internal.h"

namespace hisq {
hisq_status check_gauge(hisq_gauge g);
hisq_status check_vec(const void *p, const char *name);
hisq_status check_nrhs(int nrhs);
hisq_status check_mass(double two_m, bool positive);
}  // namespace hisq

using namespace hisq;

namespace {

constexpr size_t kScratchBytes = HISQ_NOALLOC_SCRATCH_BYTES;

// One copy per GPU, at its own address on each.  In host code the name is a
// host-side stand-in: kernels get the device address from
// hipGetSymbolAddress, kept per device below.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per
// device, with that device current).
hisq_status scratch_address(int device, void **out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(HISQ_ERR_INVALID_ARG, "hisq_mdagm_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HISQ_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return HISQ_OK;
}

}  // namespace

extern "C" hisq_status hisq_mdagm_noalloc(hisq_gauge g, double two_m, const void *in_e_dev,
                                          void *out_e_dev, int nrhs, hisq_prec prec,
                                          void *stream) {
    HISQ_TRY(check_gauge(g));
    HISQ_TRY(check_nrhs(nrhs));
    HISQ_TRY(check_mass(two_m, false));
    HISQ_TRY(check_vec(in_e_dev, "in_e_dev"));
    HISQ_TRY(check_vec(out_e_dev, "out_e_dev"));
    if (in_e_dev == out_e_dev) return fail(HISQ_ERR_INVALID_ARG, "in and out must not overlap");
    if (prec != HISQ_FP64 && prec != HISQ_FP32)
        return fail(HISQ_ERR_INVALID_ARG, "hisq_mdagm_noalloc: prec must be HISQ_FP64 or HISQ_FP32");
    if (prec == HISQ_FP32 && !g->fat32[0])
        return fail(HISQ_ERR_INVALID_ARG,
                    "hisq_mdagm_noalloc: the FP32 links of this handle do not exist yet (a "
                    "hisq_mdagm or hisq_dslash_eo call with HISQ_FP32 makes them)");
    const size_t per = prec == HISQ_FP64 ? sizeof(double2) : sizeof(float2);
    const size_t need = per * 3 * (size_t)g->geom.vh * (size_t)nrhs;
    if (need > kScratchBytes)
        return fail(HISQ_ERR_INVALID_ARG,
                    "hisq_mdagm_noalloc: the odd temporary needs " + std::to_string(need) +
                        " bytes, more than the " + std::to_string(kScratchBytes) +
                        " of the allocation-free scratch (use hisq_mdagm, or fewer RHS)");
    int device = -1;
    HISQ_HIP(hipGetDevice(&device));
    if (device != g->device)
        return fail(HISQ_ERR_INVALID_ARG,
                    "hisq_mdagm_noalloc: the current device is not the handle's device");
    void *t = nullptr;
    HISQ_TRY(scratch_address(device, &t));
    const ProfileSuppress no_events;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (prec == HISQ_FP32) {
        const float2 *in = static_cast<const float2 *>(in_e_dev);
        float2 *out = static_cast<float2 *>(out_e_dev);
        float2 *tmp = static_cast<float2 *>(t);
        HISQ_TRY(launch_dslash_f32(g, 1, in, tmp, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, nullptr, s));
        return launch_dslash_f32(g, 0, tmp, out, nrhs, in, two_m * two_m, nullptr, 0.0, -1.0,
                                 nullptr, s);
    }
    const double2 *in = static_cast<const double2 *>(in_e_dev);
    double2 *out = static_cast<double2 *>(out_e_dev);
    double2 *tmp = static_cast<double2 *>(t);
    HISQ_TRY(launch_dslash(g, 1, in, tmp, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE, nullptr,
                           nullptr, s));
    return launch_dslash(g, 0, tmp, out, nrhs, in, two_m * two_m, nullptr, 0.0, -1.0, FIN_NONE,
                         nullptr, nullptr, s);
}
