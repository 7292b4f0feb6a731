// The HISQ half stencil kernel, generic in the storage precision R (double or
// float; arithmetic in R, the <aux, out> partials of the CG always in double).
//
//   out(x) = ca * aux(x) + cb * aux2(x) + cd * sum_mu [ F_mu(x) in(x+mu) - F_mu(x-mu)^H in(x-mu)
//                                                   + L_mu(x) in(x+3mu) - L_mu(x-3mu)^H in(x-3mu) ]
//
// for every site x of parity p (arXiv:2502.00152, section 2: the HISQ matrix
// D of M = D + 2m; the even-odd split makes D map one parity to the other).
//
// One thread owns one output site and NR right-hand sides.  Forward links are
// read at the thread's own checkerboard index (coalesced); backward links are
// read at the neighbour's index in the other parity's array, which is
// coalesced too for y, z, t hops (constant offset) and nearly so for x hops.
// The HBM traffic per output site is 16 links + (in + out) per RHS, so the
// kernel is bound by HBM bandwidth.  Included by dslash.hip (FP64) and
// dslash_f32.hip (FP32) only.
#pragma once

#include "device_util.h"
#include "hisq_internal.h"

namespace hisq {

template <typename R>
using vec2 = R __attribute__((ext_vector_type(2)));

namespace dslash_impl {

constexpr int kBS = 256;

template <typename R>
struct DslashArgs {
    const vec2<R> *fat_out;  // links on output-parity sites  [4][9][Vh]
    const vec2<R> *fat_in;   // links on input-parity sites   [4][9][Vh]
    const vec2<R> *lng_out;
    const vec2<R> *lng_in;
    const vec2<R> *in;       // [nrhs][3][Vh], parity 1-p
    vec2<R> *out;            // [nrhs][3][Vh], parity p
    const vec2<R> *aux;      // [nrhs][3][Vh], parity p (optional)
    const vec2<R> *aux2;     // [nrhs][3][Vh], parity p (optional; may alias out)
    R ca, cb, cd;
    Geom geom;
    int out_parity;
    int xcd_remap;         // 1: contiguous site ranges per XCD
    int group_outer;       // 1: block index = group * nsb + site block
    int nrhs;
    int ngroups;           // ceil(nrhs / NR)
    int nsb;               // site blocks
    // fused reduction (FIN_CG_ALPHA)
    double *partials;      // [nrhs][nsb]
};

__device__ __forceinline__ int wrap(int c, int L) {
    c = c < 0 ? c + L : c;
    c = c < 0 ? c + L : c;
    c = c >= L ? c - L : c;
    c = c >= L ? c - L : c;
    return c;
}

// Link loads: non-temporal when a launch reads each link once (one RHS group:
// the links should not evict the input field), plain when several RHS groups
// read the same links (L2 then serves the later groups).  The choice is a
// template argument: a runtime select lets the compiler merge the two loads
// into one plain load.
template <bool NT, typename V>
__device__ __forceinline__ V ldlink(const V *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int NR, bool NT, typename R>
__device__ __forceinline__ void hop_forward(const vec2<R> *__restrict__ U, int vh, int cbU,
                                            const vec2<R> *__restrict__ in, int64_t rstride,
                                            int cbN, int nr, vec2<R> (&acc)[NR][3]) {
    using V = vec2<R>;
    V u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = ldlink<NT>(U + (int64_t)k * vh + cbU);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r < nr) {
            const V *v = in + r * rstride + cbN;
            const V v0 = v[0], v1 = v[vh], v2 = v[2 * (int64_t)vh];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                V s = acc[r][a];
                s.x = fma(u[3 * a].x, v0.x, s.x);  s.x = fma(-u[3 * a].y, v0.y, s.x);
                s.y = fma(u[3 * a].x, v0.y, s.y);  s.y = fma(u[3 * a].y, v0.x, s.y);
                s.x = fma(u[3 * a + 1].x, v1.x, s.x);  s.x = fma(-u[3 * a + 1].y, v1.y, s.x);
                s.y = fma(u[3 * a + 1].x, v1.y, s.y);  s.y = fma(u[3 * a + 1].y, v1.x, s.y);
                s.x = fma(u[3 * a + 2].x, v2.x, s.x);  s.x = fma(-u[3 * a + 2].y, v2.y, s.x);
                s.y = fma(u[3 * a + 2].x, v2.y, s.y);  s.y = fma(u[3 * a + 2].y, v2.x, s.y);
                acc[r][a] = s;
            }
        }
    }
}

// acc -= U^H v, with U read at the neighbour's index.
template <int NR, bool NT, typename R>
__device__ __forceinline__ void hop_backward(const vec2<R> *__restrict__ U, int vh, int cbN,
                                             const vec2<R> *__restrict__ in, int64_t rstride,
                                             int nr, vec2<R> (&acc)[NR][3]) {
    using V = vec2<R>;
    V u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = ldlink<NT>(U + (int64_t)k * vh + cbN);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r < nr) {
            const V *v = in + r * rstride + cbN;
            const V v0 = v[0], v1 = v[vh], v2 = v[2 * (int64_t)vh];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                // (U^H)_{ab} = conj(U_{ba})
                V s = acc[r][a];
                s.x = fma(-u[a].x, v0.x, s.x);  s.x = fma(-u[a].y, v0.y, s.x);
                s.y = fma(-u[a].x, v0.y, s.y);  s.y = fma(u[a].y, v0.x, s.y);
                s.x = fma(-u[3 + a].x, v1.x, s.x);  s.x = fma(-u[3 + a].y, v1.y, s.x);
                s.y = fma(-u[3 + a].x, v1.y, s.y);  s.y = fma(u[3 + a].y, v1.x, s.y);
                s.x = fma(-u[6 + a].x, v2.x, s.x);  s.x = fma(-u[6 + a].y, v2.y, s.x);
                s.y = fma(-u[6 + a].x, v2.y, s.y);  s.y = fma(u[6 + a].y, v2.x, s.y);
                acc[r][a] = s;
            }
        }
    }
}

template <typename R, int NR, bool AUX, bool AUX2, bool DOT, bool NT>
__global__ __launch_bounds__(kBS) void k_dslash(DslashArgs<R> a) {
    using V = vec2<R>;
    const Geom g = a.geom;
    const int vh = g.vh;
    const int lb = a.xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    int sb, grp;
    if (a.group_outer) {
        grp = lb / a.nsb;
        sb = lb - grp * a.nsb;
    } else {
        sb = lb / a.ngroups;
        grp = lb - sb * a.ngroups;
    }
    const int cb = sb * kBS + threadIdx.x;
    const int r0 = grp * NR;
    const int nr = min(NR, a.nrhs - r0);
    const int64_t rstride = 3 * (int64_t)vh;

    double dotv[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) dotv[r] = 0.0;

    if (cb < vh) {
        // coordinates of the output site
        int t = cb / g.Xh;
        const int xh = cb - t * g.Xh;
        const int y = t % g.Y;
        t /= g.Y;
        const int z = t % g.Z;
        t /= g.Z;
        const int x = 2 * xh + ((a.out_parity + y + z + t) & 1);
        const int rowYZT = (t * g.Z + z) * g.Y + y;  // lex = rowYZT * X + x

        V acc[NR][3];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[r][c] = V{R(0), R(0)};

        const V *in = a.in + r0 * rstride;
        const int64_t lstride = 9 * (int64_t)vh;

#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int hop = h == 0 ? 1 : 3;
            const V *Uo = h == 0 ? a.fat_out : a.lng_out;
            const V *Ui = h == 0 ? a.fat_in : a.lng_in;
            // mu = 0 (x)
            {
                const int f = (rowYZT * g.X + wrap(x + hop, g.X)) >> 1;
                const int b = (rowYZT * g.X + wrap(x - hop, g.X)) >> 1;
                hop_forward<NR, NT, R>(Uo, vh, cb, in, rstride, f, nr, acc);
                hop_backward<NR, NT, R>(Ui, vh, b, in, rstride, nr, acc);
            }
            // mu = 1 (y)
            {
                const int f = ((((t * g.Z + z) * g.Y + wrap(y + hop, g.Y)) * g.X) + x) >> 1;
                const int b = ((((t * g.Z + z) * g.Y + wrap(y - hop, g.Y)) * g.X) + x) >> 1;
                hop_forward<NR, NT, R>(Uo + lstride, vh, cb, in, rstride, f, nr, acc);
                hop_backward<NR, NT, R>(Ui + lstride, vh, b, in, rstride, nr, acc);
            }
            // mu = 2 (z)
            {
                const int f = ((((t * g.Z + wrap(z + hop, g.Z)) * g.Y + y) * g.X) + x) >> 1;
                const int b = ((((t * g.Z + wrap(z - hop, g.Z)) * g.Y + y) * g.X) + x) >> 1;
                hop_forward<NR, NT, R>(Uo + 2 * lstride, vh, cb, in, rstride, f, nr, acc);
                hop_backward<NR, NT, R>(Ui + 2 * lstride, vh, b, in, rstride, nr, acc);
            }
            // mu = 3 (t)
            {
                const int f = ((((wrap(t + hop, g.T) * g.Z + z) * g.Y + y) * g.X) + x) >> 1;
                const int b = ((((wrap(t - hop, g.T) * g.Z + z) * g.Y + y) * g.X) + x) >> 1;
                hop_forward<NR, NT, R>(Uo + 3 * lstride, vh, cb, in, rstride, f, nr, acc);
                hop_backward<NR, NT, R>(Ui + 3 * lstride, vh, b, in, rstride, nr, acc);
            }
        }

        // epilogue
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r < nr) {
                const int64_t base = (r0 + r) * rstride + cb;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    V o = acc[r][c] * a.cd;
                    if (AUX) {
                        const V ax = a.aux[base + c * (int64_t)vh];
                        o.x = fma(a.ca, ax.x, o.x);
                        o.y = fma(a.ca, ax.y, o.y);
                        if (AUX2) {
                            const V a2 = a.aux2[base + c * (int64_t)vh];
                            o.x = fma(a.cb, a2.x, o.x);
                            o.y = fma(a.cb, a2.y, o.y);
                        }
                        if (DOT)
                            dotv[r] = fma((double)ax.x, (double)o.x,
                                          fma((double)ax.y, (double)o.y, dotv[r]));
                    }
                    a.out[base + c * (int64_t)vh] = o;
                }
            }
        }
    }

    if (DOT) {
        // per-block partial sums of Re<aux, out>; the CG update kernel adds them
        // up in block order (no cross-block synchronisation in this kernel)
        __shared__ double lds[NR * (kBS / kWave)];
        block_sum<NR, kBS>(dotv, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r < nr) a.partials[(int64_t)(r0 + r) * a.nsb + sb] = dotv[r];
        }
    }
}

template <typename R, int NR, bool NT>
void launch_variant(const DslashArgs<R> &args, int nblocks, bool aux, bool aux2, bool dot,
                    hipStream_t s) {
    if (dot)
        hipLaunchKernelGGL((k_dslash<R, NR, true, false, true, NT>), dim3(nblocks), dim3(kBS), 0, s,
                           args);
    else if (aux2)
        hipLaunchKernelGGL((k_dslash<R, NR, true, true, false, NT>), dim3(nblocks), dim3(kBS), 0, s,
                           args);
    else if (aux)
        hipLaunchKernelGGL((k_dslash<R, NR, true, false, false, NT>), dim3(nblocks), dim3(kBS), 0, s,
                           args);
    else
        hipLaunchKernelGGL((k_dslash<R, NR, false, false, false, NT>), dim3(nblocks), dim3(kBS), 0,
                           s, args);
}

template <typename R, int NR>
hisq_status launch_nr(const DslashArgs<R> &args, int nblocks, bool aux, bool aux2, bool dot,
                      hipStream_t s) {
    if (args.ngroups == 1)
        launch_variant<R, NR, true>(args, nblocks, aux, aux2, dot, s);
    else
        launch_variant<R, NR, false>(args, nblocks, aux, aux2, dot, s);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

// Fill the argument block and launch with NR right-hand sides per thread.
template <typename R>
hisq_status launch_dslash_t(const Geom &geom, const vec2<R> *const fat[2],
                            const vec2<R> *const lng[2], int out_parity, const vec2<R> *in,
                            vec2<R> *out, int nrhs, const vec2<R> *aux, double ca,
                            const vec2<R> *aux2, double cb, double cd, double *partials, int nr,
                            int xcd_remap, int group_outer, hipStream_t s) {
    if (aux2 && !aux) return fail(HISQ_ERR_INVALID_ARG, "dslash: aux2 needs aux");
    DslashArgs<R> a{};
    const int p = out_parity;
    a.fat_out = fat[p];
    a.fat_in = fat[1 - p];
    a.lng_out = lng[p];
    a.lng_in = lng[1 - p];
    a.in = in;
    a.out = out;
    a.aux = aux;
    a.aux2 = aux2;
    a.ca = (R)ca;
    a.cb = (R)cb;
    a.cd = (R)cd;
    a.geom = geom;
    a.out_parity = p;
    a.xcd_remap = xcd_remap;
    a.group_outer = group_outer;
    a.nrhs = nrhs;
    a.ngroups = (nrhs + nr - 1) / nr;
    a.nsb = (geom.vh + kBS - 1) / kBS;
    a.partials = partials;
    const bool dot = partials != nullptr;
    const int nblocks = a.nsb * a.ngroups;
    switch (nr) {
        case 1: return launch_nr<R, 1>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 2: return launch_nr<R, 2>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 3: return launch_nr<R, 3>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 4: return launch_nr<R, 4>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 6: return launch_nr<R, 6>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 12: return launch_nr<R, 12>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        default: return fail(HISQ_ERR_INVALID_ARG, "dslash: bad RHS grouping");
    }
}


}  // namespace dslash_impl
}  // namespace hisq
