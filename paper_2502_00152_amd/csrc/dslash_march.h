// The multi-RHS half stencil for large volumes, marching along time.
//
// Same operator, same hop order and arithmetic, same epilogue and the same
// canonical <aux, out> partials as k_dslash (dslash_kernel.h), so its output
// is bitwise that of k_dslash; only the order in which sites are visited
// differs.
//
// Why.  At volumes beyond the last-level cache the standard kernel visits the
// sites of a parity in checkerboard order; the time neighbours of a site are
// a whole time slice away (Xh Y Z sites), and with several RHS per site the
// sites in flight on one XCD carry more data than its 4 MB L2, so each input
// site is fetched from beyond L2 many times (measured on 48^3 x 96 with 12
// RHS: 2.7x the algorithmic bytes with 16-bit vectors, 4.4x with FP32).
//
// Work decomposition.  Checkerboard index cb = t S + j with S = Xh Y Z sites
// per time slice and parity, and j = (z Y + y) Xh + xh.  For fixed j the
// output sites at t and t + 2 sit on the same lattice column (x, y, z), and
// their time neighbours t +- 1, t +- 3 are the input sites t' S + j of that
// column.  A workgroup owns kSites consecutive j (one canonical partial-sum
// chunk of every slice it visits) for one slice parity s and one RHS group,
// and marches over the output slices t = 2k + s of one time segment.  Each
// lane keeps the input at t - 3, t - 1, t + 1, t + 3 of its column in
// registers (a ring; one new slice is loaded per step), so the
// four time hops of a site read no memory beyond their links; the x, y and z
// neighbours of slice t are gathered as in k_dslash, from data that the
// workgroups of neighbouring chunks loaded into L2 a step or two earlier.
// Block order: (segment, chunk, group, s) with s fastest, so both slice
// parities and all RHS groups of a chunk run side by side, and each XCD
// takes a contiguous range of chunks.
#pragma once

#include "dslash_kernel.h"

namespace hisq {
namespace dslash_impl {

struct MarchGeo {
    int S;       // sites per time slice and parity (Xh Y Z), a multiple of kSites
    int nchunk;  // S / kSites
    int nseg;    // time segments
    int kseg;    // march steps per segment (the last segment may be shorter)
    int nsteps;  // T / 2
};

// The neighbour vectors of one lattice column slice: the stored values (for
// packed 16-bit vectors, the three colours and the norm of each RHS).
template <int NR, typename VS>
struct RingSlot {
    using E = typename std::conditional<is_normed<VS>(), h16c, VS>::type;
    E v[NR][3];
    float n[NR];
};

template <int NR, typename VS>
__device__ __forceinline__ void march_load_vec(RingSlot<NR, VS> &d, const VS *__restrict__ in,
                                               int vh, uint32_t voff,
                                               const uint32_t (&roff)[NR]) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if constexpr (is_normed<VS>()) {
            h16_unpack(*at(in, roff[r] + voff), d.v[r], d.n[r]);
        } else {
            d.v[r][0] = *at(in, roff[r] + voff);
            d.v[r][1] = *at(in + vh, roff[r] + voff);
            d.v[r][2] = *at(in + 2 * (int64_t)vh, roff[r] + voff);
        }
    }
}

// The raw operands of one hop (links and the neighbour's vectors).
template <typename R, typename VS, typename LS, int NR>
struct MarchRaw {
    static constexpr bool kInt = int_hops<VS, LS>();
    using Raw = typename std::conditional<kInt, HopRaw<NR>, HopRawG<NR, VS, LS>>::type;
};

// The link at byte offset uoff of one direction (lstride words per direction).
template <bool NT, typename LS, typename UT>
__device__ __forceinline__ void march_load_links(UT (&u)[9], const LS *__restrict__ U,
                                                 int64_t lstride, uint32_t uoff) {
    if constexpr (std::is_same<LS, q16s>::value) {
        load_link_q16s<NT>(u, U, lstride / 9, uoff);
    } else {
        const gptr<const LS> up = at(U, uoff);
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] = ldlink<NT>(up + k * kLinkTile);
    }
}

template <typename R, typename VS, typename LS, int NR, bool FWD, typename Raw>
__device__ __forceinline__ void march_math(const Raw &d, vec2<R> (&acc)[NR][3]) {
    if constexpr (int_hops<VS, LS>()) hop_math<NR, FWD>(d, acc);
    else hop_math_g<NR, FWD, R>(d, acc);
}

// Hops of lookahead per shape: none for the register-heavy shapes (6 RHS
// per lane, or 4 lanes per site with their 128-register cap).
constexpr int march_lookahead(int nr, int lps) { return (nr >= 6 || lps >= 4) ? 0 : 1; }

template <typename R, typename VS, typename LS, int NR, int LPS, bool AUX, bool AUX2, bool DOT,
          bool NT>
__global__ __launch_bounds__(kSites *LPS) void k_dslash_march(DslashArgs<R, VS, LS> a,
                                                              MarchGeo mg) {
    using V = vec2<R>;
    using Raw = typename MarchRaw<R, VS, LS, NR>::Raw;
    constexpr int SPW = kWave / LPS;  // sites per wave
    constexpr int RG = LPS * NR;      // RHS per group
    const Geom g = a.geom;
    const int vh = g.vh;
    const int lb = remap_block(a.xcd_remap, (int)blockIdx.x, (int)gridDim.x);
    const int s = lb & 1;
    int rest = lb >> 1;
    const int grp = rest % a.ngroups;
    rest /= a.ngroups;
    const int c = rest % mg.nchunk;
    const int sg = rest / mg.nchunk;
    const int k0 = sg * mg.kseg;
    const int k1 = min(k0 + mg.kseg, mg.nsteps);
    const int w = threadIdx.x / kWave, l = threadIdx.x & (kWave - 1);
    const int q = l / SPW;                   // RHS slot of this lane
    const int sl = w * SPW + (l - q * SPW);  // site within the chunk
    const int j = c * kSites + sl;           // index within a time slice
    const int rg0 = grp * RG;
    const int nr = min(NR, a.nrhs - rg0 - q * NR);
    constexpr int CP = planes<VS>();
    const uint32_t qoff = (uint32_t)(q * NR * CP) * (uint32_t)vh * (uint32_t)sizeof(VS);
    const int cps = mg.S / kSites;  // chunks per slice

    if (a.rhs_status) {
        bool any = false;
        for (int r = rg0; r < min(rg0 + RG, a.nrhs); ++r) any = any || a.rhs_status[r] == CG_ACTIVE;
        if (!any) {
            if (DOT && threadIdx.x < RG && rg0 + (int)threadIdx.x < a.nrhs)
                for (int k = k0; k < k1; ++k)
                    a.partials[(int64_t)(rg0 + threadIdx.x) * a.nsb + (2 * k + s) * cps + c] = 0.0;
            return;
        }
    }

    // the lattice column of this lane: x is the same at every output slice
    // t = s (mod 2)
    const int xh = j % g.Xh;
    const int yz = j / g.Xh;
    const int y = yz % g.Y;
    const int z = yz / g.Y;
    const int x = 2 * xh + ((a.out_parity + y + z + s) & 1);
    const bool live = nr > 0;

    // the group's first RHS exists (rg0 < nrhs); a lane past the last RHS of
    // a ragged group reads that first RHS's planes and stores nothing
    const VS *in = a.in + (int64_t)rg0 * CP * vh;
    uint32_t roff[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r)
        roff[r] = live ? qoff + (uint32_t)(CP * min(r, nr - 1)) * (uint32_t)vh * (uint32_t)sizeof(VS)
                       : 0u;
    const int64_t lstride = 9 * kLinkTile * link_tiles(vh);
    const VS *const in_l = in;

    auto slice = [&](int t) {
        t %= g.T;
        return t < 0 ? t + g.T : t;
    };
    auto vcol = [&](int t) { return (uint32_t)(slice(t) * mg.S + j) * (uint32_t)sizeof(VS); };

    // inputs at t-3, t-1, t+1, t+3; slot 3 is loaded at the start of each step
    // (its first use, the long forward time hop, comes fourteen hops later)
    RingSlot<NR, VS> ring[4];
    {
        const int t0 = 2 * k0 + s;
        march_load_vec<NR>(ring[0], in_l, vh, vcol(t0 - 3), roff);
        march_load_vec<NR>(ring[1], in_l, vh, vcol(t0 - 1), roff);
        march_load_vec<NR>(ring[2], in_l, vh, vcol(t0 + 1), roff);
    }

    const LS *const Uo[2] = {a.fat_out, a.lng_out};
    const LS *const Ui[2] = {a.fat_in, a.lng_in};
    __shared__ double red[DOT ? RG * kSites : 1];

    for (int k = k0; k < k1; ++k) {
        const int t = 2 * k + s;
        march_load_vec<NR>(ring[3], in_l, vh, vcol(t + 3), roff);
        const int cb = slice(t) * mg.S + j;
        const uint32_t own_l = link_off<LS>(cb);

        V acc[NR][3];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) acc[r][cc] = V{R(0), R(0)};

        // the 16 hops in the order of k_dslash (fat then long; x, y, z, t;
        // forward then backward); the time hops take their vectors from the ring
        auto load = [&](int i, Raw &d) {
            const int h = i >> 3, mu = (i >> 1) & 3;
            const int dist = h == 0 ? 1 : 3;
            const bool fwd = (i & 1) == 0;
            if (mu == 3) {
                const int b = slice(t - dist) * mg.S + j;
                if (fwd) march_load_links<NT, LS>(d.u, Uo[h] + mu * lstride, lstride, own_l);
                else march_load_links<NT, LS>(d.u, Ui[h] + mu * lstride, lstride, link_off<LS>(b));
                const RingSlot<NR, VS> &rs = ring[fwd ? (h == 0 ? 2 : 3) : (h == 0 ? 1 : 0)];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) d.v[r][cc] = rs.v[r][cc];
                    if constexpr (is_normed<VS>()) d.n[r] = rs.n[r];
                }
            } else {
                const int nb = nbr_cb(g, x, y, z, slice(t), mu, fwd ? dist : -dist);
                if (fwd) march_load_links<NT, LS>(d.u, Uo[h] + mu * lstride, lstride, own_l);
                else march_load_links<NT, LS>(d.u, Ui[h] + mu * lstride, lstride, link_off<LS>(nb));
                RingSlot<NR, VS> tmp;
                march_load_vec<NR>(tmp, in_l, vh, (uint32_t)nb * (uint32_t)sizeof(VS), roff);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) d.v[r][cc] = tmp.v[r][cc];
                    if constexpr (is_normed<VS>()) d.n[r] = tmp.n[r];
                }
            }
        };
        // one hop of lookahead (the next hop's loads issued before this hop's
        // arithmetic) where the registers allow it
        constexpr int LA = march_lookahead(NR, LPS);
        Raw buf[LA + 1];
#pragma unroll
        for (int i = 0; i < LA; ++i) load(i, buf[i]);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i + LA < 16) load(i + LA, buf[(i + LA) % (LA + 1)]);
            if ((i & 1) == 0) march_math<R, VS, LS, NR, true>(buf[i % (LA + 1)], acc);
            else march_math<R, VS, LS, NR, false>(buf[i % (LA + 1)], acc);
            hop_fence<NR>(acc);
        }

        // epilogue, as in k_dslash
        double dotv[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) dotv[r] = 0.0;
        const uint32_t own = (uint32_t)cb * (uint32_t)sizeof(VS);
        if (live) {
            if constexpr (is_normed<VS>()) {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (r < nr) {
                        const R ca = AUX ? (a.ca_rhs ? (R)a.ca_rhs[rg0 + q * NR + r] : a.ca) : R(0);
                        h16_epilogue<AUX, DOT>(acc[r], a.cd, ca, a.aux + (int64_t)(rg0 + r) * vh,
                                               a.out + (int64_t)(rg0 + r) * vh, qoff + own, dotv[r]);
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if (r < nr) {
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) {
                            const int64_t plane = (int64_t)(rg0 * 3 + 3 * r + cc) * vh;
                            const uint32_t off = qoff + own;
                            V o = acc[r][cc] * a.cd;
                            if (AUX) {
                                const V ax = Conv<VS>::template ld<R>(*at(a.aux + plane, off));
                                const R ca = a.ca_rhs ? (R)a.ca_rhs[rg0 + q * NR + r] : a.ca;
                                o.x = fma(ca, ax.x, o.x);
                                o.y = fma(ca, ax.y, o.y);
                                if (AUX2) {
                                    const V a2 = Conv<VS>::template ld<R>(*at(a.aux2 + plane, off));
                                    o.x = fma(a.cb, a2.x, o.x);
                                    o.y = fma(a.cb, a2.y, o.y);
                                }
                                if (DOT)
                                    dotv[r] = fma((double)ax.x, (double)o.x,
                                                  fma((double)ax.y, (double)o.y, dotv[r]));
                            }
                            *at(a.out + plane, off) = Conv<VS>::template st<R>(o);
                        }
                    }
                }
            }
        }
        if (DOT) {
            // the canonical partial of this slice's chunk, as k_dslash forms it
#pragma unroll
            for (int r = 0; r < NR; ++r) red[(q * NR + r) * kSites + sl] = dotv[r];
            __syncthreads();
            constexpr int NW = kSites * LPS / kWave;
            for (int jj = w; jj < RG; jj += NW) {
                const double sm = chunk_sum(red + jj * kSites);
                if (l == 0 && rg0 + jj < a.nrhs)
                    a.partials[(int64_t)(rg0 + jj) * a.nsb + slice(t) * cps + c] = sm;
            }
            __syncthreads();
        }
        // advance the ring: t+2 needs t-1, t+1, t+3 (and t+5, loaded next step)
        ring[0] = ring[1];
        ring[1] = ring[2];
        ring[2] = ring[3];
    }
}

// Launch of the marching kernel for one shape; nseg time segments.
template <typename R, typename VS, typename LS, int NR, int LPS, bool NT>
void march_variant(const DslashArgs<R, VS, LS> &args, const MarchGeo &mg, int nblocks, bool aux,
                   bool aux2, bool dot, hipStream_t s) {
    const dim3 grid(nblocks), block(kSites * LPS);
    if (dot)
        hipLaunchKernelGGL((k_dslash_march<R, VS, LS, NR, LPS, true, false, true, NT>), grid, block,
                           0, s, args, mg);
    else if (aux2)
        hipLaunchKernelGGL((k_dslash_march<R, VS, LS, NR, LPS, true, true, false, NT>), grid, block,
                           0, s, args, mg);
    else if (aux)
        hipLaunchKernelGGL((k_dslash_march<R, VS, LS, NR, LPS, true, false, false, NT>), grid,
                           block, 0, s, args, mg);
    else
        hipLaunchKernelGGL((k_dslash_march<R, VS, LS, NR, LPS, false, false, false, NT>), grid,
                           block, 0, s, args, mg);
}

template <typename R, typename VS, typename LS>
hisq_status launch_march(const DslashArgs<R, VS, LS> &a, const DslashShape &sh, bool aux,
                         bool aux2, bool dot, hipStream_t s) {
    const Geom &g = a.geom;
    MarchGeo mg{};
    mg.S = g.Xh * g.Y * g.Z;
    if (mg.S % kSites != 0 || g.T < 2)
        return fail(HISQ_ERR_INVALID_ARG, "dslash: the time-marching kernel needs Xh Y Z to be a "
                                          "multiple of 256");
    if (!march_shape_supported(march_kind<R, VS, LS>(), sh.nr, sh.lps))
        return fail(HISQ_ERR_INVALID_ARG, "dslash: shape not built for the time-marching kernel");
    mg.nchunk = mg.S / kSites;
    mg.nsteps = g.T / 2;
    const int nseg = std::max(1, std::min(sh.march, mg.nsteps));
    mg.kseg = (mg.nsteps + nseg - 1) / nseg;
    mg.nseg = (mg.nsteps + mg.kseg - 1) / mg.kseg;
    const int64_t nblocks = (int64_t)mg.nseg * mg.nchunk * a.ngroups * 2;
    if (nblocks > (int64_t)INT32_MAX) return fail(HISQ_ERR_INVALID_ARG, "dslash: grid too large");
    const bool nt = a.ngroups == 1;
#define HISQ_MARCH(NR_, LPS_)                                                                   \
    if constexpr (march_shape_supported(march_kind<R, VS, LS>(), NR_, LPS_)) {                 \
        if (sh.nr == NR_ && sh.lps == LPS_) {                                                  \
            if (nt) march_variant<R, VS, LS, NR_, LPS_, true>(a, mg, (int)nblocks, aux, aux2, dot, s); \
            else march_variant<R, VS, LS, NR_, LPS_, false>(a, mg, (int)nblocks, aux, aux2, dot, s); \
            HISQ_HIP(hipGetLastError());                                                       \
            return HISQ_OK;                                                                    \
        }                                                                                      \
    }
    HISQ_MARCH(1, 2)
    HISQ_MARCH(2, 2)
    HISQ_MARCH(3, 2)
    HISQ_MARCH(6, 2)
    HISQ_MARCH(3, 4)
#undef HISQ_MARCH
    return fail(HISQ_ERR_INVALID_ARG, "dslash: unsupported time-marching shape");
}

}  // namespace dslash_impl
}  // namespace hisq
