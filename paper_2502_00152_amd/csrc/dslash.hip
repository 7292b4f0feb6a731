// HISQ half stencil D_{p,1-p} on gfx950, FP64.
//
//   out(x) = ca * aux(x) + cb * aux2(x) + cd * sum_mu [ F_mu(x) in(x+mu) - F_mu(x-mu)^H in(x-mu)
//                                      + L_mu(x) in(x+3mu) - L_mu(x-3mu)^H in(x-3mu) ]
//
// for every site x of parity p (arXiv:2502.00152, section 2: the HISQ matrix
// D of M = D + 2m; the even-odd split makes D map one parity to the other).
//
// One thread owns one output site and NR right-hand sides.  Forward links are
// read at the thread's own checkerboard index (coalesced); backward links are
// read at the neighbour's index in the other parity's array, which is
// coalesced too for y, z, t hops (constant offset) and nearly so for x hops.
// Links are streamed with non-temporal loads: each is used once per launch,
// so they should not evict the input field, which every site reads 16 times.
// The HBM traffic per output site is 16 links * 144 B + (in + out) * 48 B * NR,
// so the kernel is bound by HBM bandwidth.
#include "device_util.h"
#include "hisq_internal.h"

namespace hisq {

typedef double dvec2 __attribute__((ext_vector_type(2)));

// Process-wide launch-shape knobs (hisq_set_tuning).
struct DslashTuning {
    int64_t rhs_per_thread = 0;
    int64_t group_order = 0;
    int64_t xcd_remap = 1;
};
DslashTuning g_tune;

namespace {

constexpr int kBS = 256;

struct DslashArgs {
    const dvec2 *fat_out;  // links on output-parity sites  [4][9][Vh]
    const dvec2 *fat_in;   // links on input-parity sites   [4][9][Vh]
    const dvec2 *lng_out;
    const dvec2 *lng_in;
    const dvec2 *in;       // [nrhs][3][Vh], parity 1-p
    dvec2 *out;            // [nrhs][3][Vh], parity p
    const dvec2 *aux;      // [nrhs][3][Vh], parity p (optional)
    const dvec2 *aux2;     // [nrhs][3][Vh], parity p (optional; may alias out)
    double ca, cb, cd;
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
template <bool NT>
__device__ __forceinline__ dvec2 ldlink(const dvec2 *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int NR, bool NT>
__device__ __forceinline__ void hop_forward(const dvec2 *__restrict__ U, int vh, int cbU,
                                            const dvec2 *__restrict__ in, int64_t rstride,
                                            int cbN, int nr, dvec2 (&acc)[NR][3]) {
    dvec2 u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = ldlink<NT>(U + (int64_t)k * vh + cbU);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r < nr) {
            const dvec2 *v = in + r * rstride + cbN;
            const dvec2 v0 = v[0], v1 = v[vh], v2 = v[2 * (int64_t)vh];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                dvec2 s = acc[r][a];
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
template <int NR, bool NT>
__device__ __forceinline__ void hop_backward(const dvec2 *__restrict__ U, int vh, int cbN,
                                             const dvec2 *__restrict__ in, int64_t rstride,
                                             int nr, dvec2 (&acc)[NR][3]) {
    dvec2 u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = ldlink<NT>(U + (int64_t)k * vh + cbN);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r < nr) {
            const dvec2 *v = in + r * rstride + cbN;
            const dvec2 v0 = v[0], v1 = v[vh], v2 = v[2 * (int64_t)vh];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                // (U^H)_{ab} = conj(U_{ba})
                dvec2 s = acc[r][a];
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

template <int NR, bool AUX, bool AUX2, bool DOT, bool NT>
__global__ __launch_bounds__(kBS) void k_dslash(DslashArgs a) {
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

        dvec2 acc[NR][3];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[r][c] = dvec2{0.0, 0.0};

        const dvec2 *in = a.in + r0 * rstride;
        const int64_t lstride = 9 * (int64_t)vh;

#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int hop = h == 0 ? 1 : 3;
            const dvec2 *Uo = h == 0 ? a.fat_out : a.lng_out;
            const dvec2 *Ui = h == 0 ? a.fat_in : a.lng_in;
            // mu = 0 (x)
            {
                const int f = (rowYZT * g.X + wrap(x + hop, g.X)) >> 1;
                const int b = (rowYZT * g.X + wrap(x - hop, g.X)) >> 1;
                hop_forward<NR, NT>(Uo, vh, cb, in, rstride, f, nr, acc);
                hop_backward<NR, NT>(Ui, vh, b, in, rstride, nr, acc);
            }
            // mu = 1 (y)
            {
                const int f = ((((t * g.Z + z) * g.Y + wrap(y + hop, g.Y)) * g.X) + x) >> 1;
                const int b = ((((t * g.Z + z) * g.Y + wrap(y - hop, g.Y)) * g.X) + x) >> 1;
                hop_forward<NR, NT>(Uo + lstride, vh, cb, in, rstride, f, nr, acc);
                hop_backward<NR, NT>(Ui + lstride, vh, b, in, rstride, nr, acc);
            }
            // mu = 2 (z)
            {
                const int f = ((((t * g.Z + wrap(z + hop, g.Z)) * g.Y + y) * g.X) + x) >> 1;
                const int b = ((((t * g.Z + wrap(z - hop, g.Z)) * g.Y + y) * g.X) + x) >> 1;
                hop_forward<NR, NT>(Uo + 2 * lstride, vh, cb, in, rstride, f, nr, acc);
                hop_backward<NR, NT>(Ui + 2 * lstride, vh, b, in, rstride, nr, acc);
            }
            // mu = 3 (t)
            {
                const int f = ((((wrap(t + hop, g.T) * g.Z + z) * g.Y + y) * g.X) + x) >> 1;
                const int b = ((((wrap(t - hop, g.T) * g.Z + z) * g.Y + y) * g.X) + x) >> 1;
                hop_forward<NR, NT>(Uo + 3 * lstride, vh, cb, in, rstride, f, nr, acc);
                hop_backward<NR, NT>(Ui + 3 * lstride, vh, b, in, rstride, nr, acc);
            }
        }

        // epilogue
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r < nr) {
                const int64_t base = (r0 + r) * rstride + cb;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    dvec2 o = acc[r][c] * a.cd;
                    if (AUX) {
                        const dvec2 ax = a.aux[base + c * (int64_t)vh];
                        o.x = fma(a.ca, ax.x, o.x);
                        o.y = fma(a.ca, ax.y, o.y);
                        if (AUX2) {
                            const dvec2 a2 = a.aux2[base + c * (int64_t)vh];
                            o.x = fma(a.cb, a2.x, o.x);
                            o.y = fma(a.cb, a2.y, o.y);
                        }
                        if (DOT) dotv[r] = fma(ax.x, o.x, fma(ax.y, o.y, dotv[r]));
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

template <int NR, bool NT>
void launch_variant(const DslashArgs &args, int nblocks, bool aux, bool aux2, bool dot,
                    hipStream_t s) {
    if (dot)
        hipLaunchKernelGGL((k_dslash<NR, true, false, true, NT>), dim3(nblocks), dim3(kBS), 0, s, args);
    else if (aux2)
        hipLaunchKernelGGL((k_dslash<NR, true, true, false, NT>), dim3(nblocks), dim3(kBS), 0, s, args);
    else if (aux)
        hipLaunchKernelGGL((k_dslash<NR, true, false, false, NT>), dim3(nblocks), dim3(kBS), 0, s, args);
    else
        hipLaunchKernelGGL((k_dslash<NR, false, false, false, NT>), dim3(nblocks), dim3(kBS), 0, s, args);
}

template <int NR>
hisq_status launch_nr(const DslashArgs &args, int nblocks, bool aux, bool aux2, bool dot,
                      hipStream_t s) {
    if (args.ngroups == 1)
        launch_variant<NR, true>(args, nblocks, aux, aux2, dot, s);
    else
        launch_variant<NR, false>(args, nblocks, aux, aux2, dot, s);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

// Right-hand sides per thread: the tuned value, else measured defaults.  With
// many RHS the input field no longer fits the per-XCD L2 and the neighbour
// gathers are served from the last-level cache; then occupancy (latency
// hiding) matters more than link reuse in registers: 2 per thread up to
// Vh = 2^18 (16^3 x 32 with 12 RHS: 78 us against 93 us with 4), 3 above
// (32^3 x 64: 1.68 ms against 1.74 ms).  A group may be partly empty; lanes
// mask r < nr.
int pick_nr(int nrhs, int vh) {
    if (g_tune.rhs_per_thread > 0) return (int)g_tune.rhs_per_thread;
    if (nrhs <= 2) return nrhs;
    if (nrhs <= 4) return nrhs;
    return vh <= (1 << 18) ? 2 : 3;
}

}  // namespace

hisq_status dslash_set_tuning(const std::string &key, int64_t v) {
    if (key == "dslash_rhs_per_thread") {
        if (!(v == 0 || v == 1 || v == 2 || v == 3 || v == 4 || v == 6 || v == 12))
            return fail(HISQ_ERR_INVALID_ARG, "dslash_rhs_per_thread must be 0, 1, 2, 3, 4, 6 or 12");
        g_tune.rhs_per_thread = v;
    } else if (key == "dslash_group_order") {
        if (v != 0 && v != 1) return fail(HISQ_ERR_INVALID_ARG, "dslash_group_order must be 0 or 1");
        g_tune.group_order = v;
    } else if (key == "dslash_xcd_remap") {
        if (v != 0 && v != 1) return fail(HISQ_ERR_INVALID_ARG, "dslash_xcd_remap must be 0 or 1");
        g_tune.xcd_remap = v;
    } else {
        return fail(HISQ_ERR_INVALID_ARG, "unknown tuning key '" + key + "'");
    }
    return HISQ_OK;
}

int dslash_reduce_blocks(const hisq_gauge_s *g, int nrhs) {
    (void)nrhs;
    return (g->geom.vh + kBS - 1) / kBS;
}

hisq_status launch_dslash(const hisq_gauge_s *g, int out_parity, const double2 *in,
                          double2 *out, int nrhs, const double2 *aux, double ca,
                          const double2 *aux2, double cb, double cd, DslashFinal fin,
                          const CgDev *cg, const Reduce *red, hipStream_t s) {
    if (aux2 && !aux) return fail(HISQ_ERR_INVALID_ARG, "dslash: aux2 needs aux");
    DslashArgs a{};
    const int p = out_parity;
    a.fat_out = reinterpret_cast<const dvec2 *>(g->fat[p]);
    a.fat_in = reinterpret_cast<const dvec2 *>(g->fat[1 - p]);
    a.lng_out = reinterpret_cast<const dvec2 *>(g->lng[p]);
    a.lng_in = reinterpret_cast<const dvec2 *>(g->lng[1 - p]);
    a.in = reinterpret_cast<const dvec2 *>(in);
    a.out = reinterpret_cast<dvec2 *>(out);
    a.aux = reinterpret_cast<const dvec2 *>(aux);
    a.aux2 = reinterpret_cast<const dvec2 *>(aux2);
    a.ca = ca;
    a.cb = cb;
    a.cd = cd;
    a.geom = g->geom;
    a.out_parity = p;
    a.nrhs = nrhs;
    a.xcd_remap = (int)g_tune.xcd_remap;
    a.group_outer = (int)g_tune.group_order;
    const int nr = pick_nr(nrhs, g->geom.vh);
    a.ngroups = (nrhs + nr - 1) / nr;
    a.nsb = (g->geom.vh + kBS - 1) / kBS;
    const bool dot = fin == FIN_CG_ALPHA;
    (void)cg;
    if (dot) a.partials = red->partials;
    const int nblocks = a.nsb * a.ngroups;
    ProfileScope prof(aux2 ? "dslash_aux2" : aux ? "dslash_aux" : "dslash", s);
    switch (nr) {
        case 1: return launch_nr<1>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 2: return launch_nr<2>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 3: return launch_nr<3>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 4: return launch_nr<4>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 6: return launch_nr<6>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        case 12: return launch_nr<12>(a, nblocks, aux != nullptr, aux2 != nullptr, dot, s);
        default: return fail(HISQ_ERR_INVALID_ARG, "dslash: bad RHS grouping");
    }
}

hisq_status apply_mdagm(hisq_gauge_s *g, double two_m, const double2 *in, double2 *out,
                        int nrhs, hipStream_t s) {
    void *tmp = nullptr;
    HISQ_TRY(g->ws.get("mdagm_tmp", sizeof(double2) * 3 * (size_t)g->geom.vh * nrhs, &tmp));
    double2 *t = static_cast<double2 *>(tmp);
    HISQ_TRY(launch_dslash(g, 1, in, t, nrhs, nullptr, 0.0, nullptr, 0.0, 1.0, FIN_NONE,
                           nullptr, nullptr, s));
    HISQ_TRY(launch_dslash(g, 0, t, out, nrhs, in, two_m * two_m, nullptr, 0.0, -1.0, FIN_NONE,
                           nullptr, nullptr, s));
    return HISQ_OK;
}

}  // namespace hisq
