// Layout conversion kernels: canonical links -> per-parity SoA with the
// staggered phases and the antiperiodic time sign folded in, and full
// canonical vectors <-> even/odd parity vectors.
#include "device_util.h"
#include "hisq_internal.h"

namespace hisq {

namespace {

constexpr int kBS = 256;

struct SiteCoords {
    int x, y, z, t, par, cb;
};

__device__ __forceinline__ SiteCoords from_lex(int lex, const Geom &g) {
    SiteCoords c;
    int r = lex;
    c.x = r % g.X;
    r /= g.X;
    c.y = r % g.Y;
    r /= g.Y;
    c.z = r % g.Z;
    c.t = r / g.Z;
    c.par = (c.x + c.y + c.z + c.t) & 1;
    c.cb = lex >> 1;
    return c;
}

// One thread per (mu, site).  canon: [4][V][9] complex; soa[p]: tiled link
// layout (link_index).
__global__ __launch_bounds__(kBS) void k_pack_links(const double2 *__restrict__ canon,
                                                    double2 *__restrict__ soa_even,
                                                    double2 *__restrict__ soa_odd, Geom g,
                                                    double coef, unsigned flags, int hop) {
    const int64_t V = 2 * (int64_t)g.vh;
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= 4 * V) return;
    const int mu = (int)(i / V);
    const int lex = (int)(i - mu * V);
    const SiteCoords c = from_lex(lex, g);
    double s = coef;
    if (flags & HISQ_GAUGE_FOLD_PHASES) {
        const int e = mu == 0 ? 0 : mu == 1 ? c.x : mu == 2 ? c.x + c.y : c.x + c.y + c.z;
        if (e & 1) s = -s;
    }
    if ((flags & HISQ_GAUGE_ANTIPERIODIC_T) && mu == 3) {
        if (((c.t + hop) / g.T) & 1) s = -s;
    }
    double2 *dst = c.par ? soa_odd : soa_even;
    const double2 *src = canon + i * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double2 v = src[k];
        v.x *= s;
        v.y *= s;
        dst[link_index(mu, k, c.cb, link_tiles(g.vh))] = v;
    }
}

// One thread per (rhs, site): full [nrhs][V][3] <-> parity [nrhs][3][Vh].
__global__ __launch_bounds__(kBS) void k_split(const double2 *__restrict__ full,
                                               double2 *__restrict__ even,
                                               double2 *__restrict__ odd, Geom g, int nrhs) {
    const int64_t V = 2 * (int64_t)g.vh;
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= nrhs * V) return;
    const int r = (int)(i / V);
    const int lex = (int)(i - r * V);
    const SiteCoords c = from_lex(lex, g);
    double2 *dst = c.par ? odd : even;
    if (!dst) return;
    const double2 *src = full + i * 3;
#pragma unroll
    for (int k = 0; k < 3; ++k) dst[((int64_t)r * 3 + k) * g.vh + c.cb] = src[k];
}

__global__ __launch_bounds__(kBS) void k_merge(const double2 *__restrict__ even,
                                               const double2 *__restrict__ odd,
                                               double2 *__restrict__ full, Geom g, int nrhs) {
    const int64_t V = 2 * (int64_t)g.vh;
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= nrhs * V) return;
    const int r = (int)(i / V);
    const int lex = (int)(i - r * V);
    const SiteCoords c = from_lex(lex, g);
    const double2 *src = c.par ? odd : even;
    double2 *dst = full + i * 3;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double2 v = make_double2(0.0, 0.0);
        if (src) v = src[((int64_t)r * 3 + k) * g.vh + c.cb];
        dst[k] = v;
    }
}

int blocks_for(int64_t n) { return (int)((n + kBS - 1) / kBS); }

}  // namespace

hisq_status launch_pack_links(const hisq_gauge_s *g, const double2 *canon, double2 *soa[2],
                              double coef, unsigned flags, bool is_long, hipStream_t s) {
    const int64_t n = 8 * (int64_t)g->geom.vh;
    hipLaunchKernelGGL(k_pack_links, dim3(blocks_for(n)), dim3(kBS), 0, s, canon, soa[0],
                       soa[1], g->geom, coef, flags, is_long ? 3 : 1);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status launch_split(const hisq_gauge_s *g, const double2 *full, double2 *even,
                         double2 *odd, int nrhs, hipStream_t s) {
    const int64_t n = 2 * (int64_t)g->geom.vh * nrhs;
    hipLaunchKernelGGL(k_split, dim3(blocks_for(n)), dim3(kBS), 0, s, full, even, odd,
                       g->geom, nrhs);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status launch_merge(const hisq_gauge_s *g, const double2 *even, const double2 *odd,
                         double2 *full, int nrhs, hipStream_t s) {
    const int64_t n = 2 * (int64_t)g->geom.vh * nrhs;
    hipLaunchKernelGGL(k_merge, dim3(blocks_for(n)), dim3(kBS), 0, s, even, odd, full,
                       g->geom, nrhs);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

}  // namespace hisq
