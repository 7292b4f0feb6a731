// The HISQ half stencil kernel, generic in the arithmetic precision R (double
// or float) and in the storage of vectors and links (complex R, or bfloat16
// pairs with float arithmetic); the <aux, out> partials of the CG are always
// double.
//
//   out(x) = ca * aux(x) + cb * aux2(x) + cd * sum_mu [ F_mu(x) in(x+mu) - F_mu(x-mu)^H in(x-mu)
//                                                   + L_mu(x) in(x+3mu) - L_mu(x-3mu)^H in(x-3mu) ]
//
// for every site x of parity p (arXiv:2502.00152, section 2: the HISQ matrix
// D of M = D + 2m; the even-odd split makes D map one parity to the other).
//
// Work decomposition.  A block covers kSites consecutive output sites
// (checkerboard index) for one group of LPS * NR right-hand sides; it has
// kSites * LPS threads.  Inside a wave, 64 / LPS consecutive sites are served
// by LPS lanes each, lane slot q holding RHS q*NR .. q*NR+NR-1 of the group.
// The LPS lanes of one site load the same link entries in the same
// instruction, so the memory pipeline fetches each link cache line once per
// wave for all LPS * NR right-hand sides; every RHS plane is still read in
// runs of 64 / LPS consecutive sites.  Forward links are read at the site's
// own index; backward links at the neighbour's index in the other parity's
// array (constant offset for y, z, t hops, nearly so for x hops).
//
// Addresses are a wave-uniform base (scalar registers: array, direction,
// colour entry, RHS) plus a 32-bit per-lane byte offset, so each load needs no
// 64-bit vector address arithmetic.  The launcher checks that the per-lane
// offsets fit 32 bits.
//
// The <aux, out> partials of one block and RHS are summed over the block's
// kSites sites in one fixed order, whatever NR and LPS are, so the CG gives
// bitwise the same iterates for any launch shape and batch size.
// Included by dslash.hip (FP64) and dslash_f32.hip (FP32) only.
#pragma once

#include <atomic>
#include <cstdint>
#include <type_traits>

#include "device_util.h"
#include "hisq_internal.h"

namespace hisq {

template <typename R>
using vec2 = R __attribute__((ext_vector_type(2)));

// One complex number stored as two bfloat16 (real part in the low half).
using bf16c = uint32_t;
// One complex number stored as two 16-bit fixed-point integers (real part in
// the low half); the value is the integer times a scale that the launcher
// folds into the stencil's coefficient cd (links only).
using q16c = int32_t;

// Conversion between a stored complex S and the arithmetic type vec2<A>.
template <typename S>
struct Conv;

template <typename R>
struct Conv<vec2<R>> {
    template <typename A>
    static __device__ __forceinline__ vec2<A> ld(vec2<R> v) {
        return vec2<A>{(A)v.x, (A)v.y};
    }
    template <typename A>
    static __device__ __forceinline__ vec2<R> st(vec2<A> v) {
        return vec2<R>{(R)v.x, (R)v.y};
    }
};

// bfloat16 <-> float: a bfloat16 is the high half of a float's bits; stores
// round to nearest, ties to even.
__host__ __device__ __forceinline__ uint32_t bf16_bits(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

template <>
struct Conv<q16c> {
    template <typename A>
    static __device__ __forceinline__ vec2<A> ld(q16c v) {
        return vec2<A>{(A)(float)(int16_t)(v & 0xffff), (A)(float)(v >> 16)};
    }
};

template <>
struct Conv<bf16c> {
    template <typename A>
    static __device__ __forceinline__ vec2<A> ld(bf16c v) {
        return vec2<A>{(A)__uint_as_float(v << 16), (A)__uint_as_float(v & 0xffff0000u)};
    }
    template <typename A>
    static __device__ __forceinline__ bf16c st(vec2<A> v) {
        return bf16_bits((float)v.x) | (bf16_bits((float)v.y) << 16);
    }
};

// One complex number in 16-bit fixed point: two int16 (real part first).
using h16c = vec2<short>;
// The colour vector of one site and RHS in 16-bit fixed point, packed in 16
// bytes: the three complex entries as int16 pairs (x, y, z) and the bits of
// a float norm (w), the largest |component| of the three.  Value = integer *
// norm / 32767 (relative accuracy ~3e-5 per site, any magnitude).  A field is
// [nrhs][Vh] of these, so one 16-byte load brings a neighbour's whole colour
// vector (three 4-byte gathers and a norm gather in a colour-plane layout).
using h16p = int __attribute__((ext_vector_type(4)));
template <typename VS>
constexpr bool is_normed() { return std::is_same<VS, h16p>::value; }
// colour planes per RHS in a field of VS: 3 ([nrhs][3][Vh]) or 1 (packed sites)
template <typename VS>
constexpr int planes() { return is_normed<VS>() ? 1 : 3; }
constexpr float kQ16 = 32767.0f;

// The int16 pair held in a 32-bit word.  The word is taken by value: a
// __builtin_bit_cast applied directly to a vector element (v.y) reads the
// vector's element 0 with this compiler.
__device__ __forceinline__ h16c as_h16c(int w) { return __builtin_bit_cast(h16c, w); }

__device__ __forceinline__ void h16_unpack(h16p v, h16c (&c)[3], float &n) {
    c[0] = as_h16c(v.x);
    c[1] = as_h16c(v.y);
    c[2] = as_h16c(v.z);
    n = __int_as_float(v.w);
}

// 16-bit fixed-point links laid out for 16-byte loads (the copy read with
// 16-bit vectors).  Per direction: entries 0-3 of every site's matrix
// ([Vhp] x 16 bytes), then entries 4-7 (the same), then entry 8 ([Vhp] x 4
// bytes), Vhp = Vh rounded up to kLinkTile; one direction takes 9 Vhp words,
// as the tiled layout does.  A link is three loads (16, 16, 4 bytes per
// lane), each contiguous over consecutive sites.
struct q16s {
    int32_t w;
};
// Fixed-point links read with 16-bit vectors: their largest integer
// component qmax is chosen per gauge field so that a row's integer L1 norm
// (sum of |Re| + |Im|) times 32767, the largest vector component, stays below
// 2^31 and the integer dot products of a link row and a colour vector cannot
// overflow.  10922 is safe for any field (6 * 10922 * 32767 < 2^31) and is the
// floor of the choice.
constexpr int kQLinkNarrow = 10922;
// hops whose loads are in flight while a hop's arithmetic runs (16-bit path)
#ifndef HISQ_INT_LOOKAHEAD
#define HISQ_INT_LOOKAHEAD 1
#endif
constexpr int kIntLookahead = HISQ_INT_LOOKAHEAD;
// the same for the other storage types, for lanes holding two or more RHS
// (measured: 12-RHS FP32 and 16-bit-link stencils 5% faster; one RHS per lane
// at 32^3 x 64 FP32 7% slower, FP64 and BF16 unchanged, so one RHS per lane
// keeps one hop at a time)
#ifndef HISQ_GEN_LOOKAHEAD
#define HISQ_GEN_LOOKAHEAD 1
#endif
constexpr int kGenLookahead = HISQ_GEN_LOOKAHEAD;
// Lookahead that fits a lane's registers for the other storage types: a hop's
// loads take (9 link entries + 3 NR vector entries [+ NR norms]) words, the
// accumulators and the widened links 6 NR + 18 reals, addresses ~40.
constexpr int gen_lookahead(int nr, int lps, int rb, int vb, int lb, bool normed) {
    if (nr < 2) return 0;
    const int buf = (9 * lb + 3 * nr * vb + (normed ? 4 * nr : 0)) / 4;
    const int cap = (512 / lps < 256 ? 512 / lps : 256) - (6 * nr + 18) * rb / 4 - 40;
    const int fit = cap / buf - 1;
    return fit < 0 ? 0 : (fit < kGenLookahead ? fit : kGenLookahead);
}
// Lookahead that still fits the registers of a lane: a block of 256 LPS lanes
// leaves 512 / LPS registers (at most 256) per lane; a hop's loads take
// 9 + 4 NR, the accumulators 6 NR, the rearranged links and addresses ~48.
constexpr int int_lookahead(int nr, int lps) {
    const int cap = (512 / lps < 256 ? 512 / lps : 256) - 6 * nr - 48;
    const int fit = cap / (9 + 4 * nr) - 1;
    return fit < 0 ? 0 : (fit < kIntLookahead ? fit : kIntLookahead);
}
// 16-bit vectors with 16-bit links: the hops run on integer dot products
template <typename VS, typename LS>
constexpr bool int_hops() {
    return std::is_same<VS, h16p>::value && std::is_same<LS, q16s>::value;
}

// Launch shape of the half stencil: NR RHS per lane, LPS lanes per site, the
// XCD-contiguous block order and the order of site blocks and RHS groups;
// march > 0 selects the kernel that marches along time (dslash_march.h) with
// that many time segments.
struct DslashShape {
    int nr;
    int lps;
    int xcd_remap;
    int group_outer;
    int march = 0;
    int blocks_per_cu = 0;  // 0: no cap
};

// Launch shape of the half stencil (tuned or default) for nrhs RHS at half
// volume vh, real_bytes per stored vector real (8, 4 or 2); q16_links: FP32
// vectors with 16-bit links (with real_bytes 2: the packed 16-bit vectors);
// plain: a launch without an epilogue field.
DslashShape dslash_pick_shape(int nrhs, int vh, size_t real_bytes, bool q16_links,
                              const Geom &geom, bool plain = false);
// XCD remap chunk (in launched blocks) of an eighth of a time slice for
// ngroups RHS groups per site block
int xcd_chunk_blocks(const Geom &geom, int ngroups);


namespace dslash_impl {

constexpr int kSites = 256;  // output sites per block (and per partial sum)
constexpr int kLdsPerCu = 160 * 1024;   // LDS of one compute unit
constexpr int kMaxBlocksPerCu = 8;      // largest block cap of a launch shape

// R: arithmetic; VS: stored complex of the vectors; LS: of the links.
template <typename R, typename VS, typename LS>
struct DslashArgs {
    const LS *fat_out;       // links on output-parity sites  [4][9][Vh]
    const LS *fat_in;        // links on input-parity sites   [4][9][Vh]
    const LS *lng_out;
    const LS *lng_in;
    const VS *in;            // [nrhs][3][Vh], parity 1-p
    VS *out;                 // [nrhs][3][Vh], parity p
    const VS *aux;           // [nrhs][3][Vh], parity p (optional)
    const VS *aux2;          // [nrhs][3][Vh], parity p (optional; may alias out)
    R ca, cb, cd;
    const double *ca_rhs;  // per-RHS ca (device, indexed by RHS), or null for ca
    const int *rhs_status; // CG state per RHS (device) or null: a block whose RHS
                           // are all inactive (converged, frozen) does nothing
    Geom geom;
    int out_parity;
    int xcd_remap;         // 0 off, 1 contiguous site ranges per XCD, n > 1 chunks
    int group_outer;       // 1: block index = group * nsb + site block
    int blocks_per_cu;     // > 0: LDS requested so that at most this many blocks share a CU
    int nrhs;
    int ngroups;           // ceil(nrhs / (LPS * NR))
    int nsb;               // site blocks = ceil(Vh / kSites)
    double *partials;      // [nrhs][nsb] (DOT)
};

__device__ __forceinline__ int wrap(int c, int L) {
    c = c < 0 ? c + L : c;
    c = c < 0 ? c + L : c;
    c = c >= L ? c - L : c;
    c = c >= L ? c - L : c;
    return c;
}

// base + byte_off with the base pinned to scalar registers: the optimiser
// cannot fold the per-lane offset into the base (which would bring back a
// 64-bit vector add per load), so the loads use the scalar-base addressing
// form with a 32-bit vector offset.
template <typename V>
__device__ __forceinline__ uint64_t sbase(V *base) {
    const uint64_t v = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <typename V>
using gptr = __attribute__((address_space(1))) V *;  // global memory

template <typename V>
__device__ __forceinline__ gptr<const V> at(const V *base, uint32_t byte_off) {
    return reinterpret_cast<gptr<const V>>(sbase(base) + byte_off);
}

template <typename V>
__device__ __forceinline__ gptr<V> at(V *base, uint32_t byte_off) {
    return reinterpret_cast<gptr<V>>(sbase(base) + byte_off);
}

// Link loads: non-temporal when a launch reads each link once (one RHS group:
// the links should not evict the input field), plain when several RHS groups
// read the same links (L2 then serves the later groups).  The choice is a
// template argument: a runtime select lets the compiler merge the two loads
// into one plain load.
template <bool NT, typename V>
__device__ __forceinline__ V ldlink(gptr<const V> p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Byte offset of entry 0 of the link of checkerboard site cb within one
// direction's tiled array (entry k follows at k * kLinkTile entries); for the
// q16s layout, the offset of the site's 16 bytes in the first two parts (a
// quarter of it in the third).
template <typename V>
__device__ __forceinline__ uint32_t link_off(int cb) {
    if constexpr (std::is_same<V, q16s>::value) return (uint32_t)cb * 16u;
    return ((uint32_t)(cb / kLinkTile) * (9 * kLinkTile) + (uint32_t)(cb % kLinkTile)) *
           (uint32_t)sizeof(V);
}

// acc += U v for the lane's RHS; U at (base U, offset uoff), v at the
// neighbour (offset voff within each colour plane of the group).
// Compiler-only fence (emits no instruction) after each hop: the hop's
// products must be complete and the next hop's loads cannot move above it.
// This bounds the register footprint - without it the compiler issues the
// loads of all 16 hops first and spills.
template <int NR, typename V>
__device__ __forceinline__ void hop_fence(V (&acc)[NR][3]) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) __asm__ __volatile__("" : "+v"(acc[r][c])::"memory");
}

// Hops with 16-bit vectors and links (forward: acc += U v; backward:
// acc -= U^H v).  Each real or imaginary part of a row of U times the colour
// vector is a sum of six int16 products, formed exactly by three two-way
// integer dot products from the link entry rearranged once per hop: forward
// Re uses (Ur, -Ui) and Im (Ui, Ur) against (vr, vi); backward, with
// (U^H)_ab = conj(U_ba), Re uses (Ur, Ui) and Im (-Ui, Ur).  The sum is
// converted to float and scaled by the neighbour's norm (the link step and
// 1/32767 are in the coefficient cd).
//
// A hop is split into its loads (HopRaw) and its arithmetic, so that the
// kernel issues the loads of the next hops before the arithmetic of the
// current one: the neighbour gathers are served from the last-level cache
// and their latency, not the ALU, bounds a wave that waits for each hop.
template <int NR>
struct HopRaw {
    h16c u[9];
    h16c v[NR][3];
    float n[NR];
};

// The link of one direction (q16s layout, vhp sites per part) at byte offset
// uoff (link_off), as its nine int16 pairs.
template <bool NT>
__device__ __forceinline__ void load_link_q16s(h16c (&u)[9], const q16s *__restrict__ U,
                                               int64_t vhp, uint32_t uoff) {
    const h16p a = ldlink<NT>(at(reinterpret_cast<const h16p *>(U), uoff));
    const h16p b = ldlink<NT>(at(reinterpret_cast<const h16p *>(U + 4 * vhp), uoff));
    const int32_t c = ldlink<NT>(at(reinterpret_cast<const int32_t *>(U + 8 * vhp), uoff >> 2));
    u[0] = as_h16c(a.x);
    u[1] = as_h16c(a.y);
    u[2] = as_h16c(a.z);
    u[3] = as_h16c(a.w);
    u[4] = as_h16c(b.x);
    u[5] = as_h16c(b.y);
    u[6] = as_h16c(b.z);
    u[7] = as_h16c(b.w);
    u[8] = as_h16c(c);
}

template <int NR, bool NT>
__device__ __forceinline__ void hop_load(HopRaw<NR> &d, const q16s *__restrict__ U, int64_t vhp,
                                         uint32_t uoff, const h16p *__restrict__ in,
                                         uint32_t voff, const uint32_t (&roff)[NR]) {
    load_link_q16s<NT>(d.u, U, vhp, uoff);
#pragma unroll
    for (int r = 0; r < NR; ++r) h16_unpack(*at(in, roff[r] + voff), d.v[r], d.n[r]);
}

template <int NR, bool FWD>
__device__ __forceinline__ void hop_math(const HopRaw<NR> &d, vec2<float> (&acc)[NR][3]) {
    h16c ure[9], uim[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        // one packed 16-bit multiply or one byte rotation each
        const h16c u = d.u[k];
        const h16c w = __builtin_shufflevector(u, u, 1, 0);
        if constexpr (FWD) {
            ure[k] = u * h16c{1, -1};
            uim[k] = w;
        } else {
            ure[k] = u;
            uim[k] = w * h16c{-1, 1};
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const float sc = FWD ? d.n[r] : -d.n[r];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // entry of (row a, column b): 3a + b forward, 3b + a (transposed) backward
            constexpr int s0 = FWD ? 1 : 3;
            const int k0 = FWD ? 3 * a : a;
            // the first product of each sum in the three-operand form (zero as
            // an inline constant; its clamp never acts, the sums fit int32)
            int re = __builtin_amdgcn_sdot2(ure[k0], d.v[r][0], 0, true);
            re = __builtin_amdgcn_sdot2(ure[k0 + s0], d.v[r][1], re, false);
            re = __builtin_amdgcn_sdot2(ure[k0 + 2 * s0], d.v[r][2], re, false);
            int im = __builtin_amdgcn_sdot2(uim[k0], d.v[r][0], 0, true);
            im = __builtin_amdgcn_sdot2(uim[k0 + s0], d.v[r][1], im, false);
            im = __builtin_amdgcn_sdot2(uim[k0 + 2 * s0], d.v[r][2], im, false);
            acc[r][a].x = fmaf(sc, (float)re, acc[r][a].x);
            acc[r][a].y = fmaf(sc, (float)im, acc[r][a].y);
        }
    }
}

// Checkerboard index of the neighbour of (x, y, z, t) at distance dist along mu.
__device__ __forceinline__ int nbr_cb(const Geom &g, int x, int y, int z, int t, int mu, int dist) {
    if (mu == 0) x = wrap(x + dist, g.X);
    else if (mu == 1) y = wrap(y + dist, g.Y);
    else if (mu == 2) z = wrap(z + dist, g.Z);
    else t = wrap(t + dist, g.T);
    return (((t * g.Z + z) * g.Y + y) * g.X + x) >> 1;
}

// The 16 hops of a site on 16-bit vectors and links, in the order of the
// generic path (fat then long; x, y, z, t; forward then backward), with the
// loads of hop i + LA issued before the arithmetic of hop i.
template <int NR, int LA, bool NT>
__device__ __forceinline__ void int_hops_all(const q16s *const (&Uo)[2], const q16s *const (&Ui)[2],
                                             int64_t lstride, const Geom &g, int x, int y, int z,
                                             int t, uint32_t own_l, const h16p *__restrict__ in,
                                             const uint32_t (&roff)[NR],
                                             vec2<float> (&acc)[NR][3]) {
    HopRaw<NR> buf[LA + 1];
    const int64_t vhp = lstride / 9;
    auto load = [&](int i, HopRaw<NR> &d) {
        const int h = i >> 3, mu = (i >> 1) & 3;
        const int dist = h == 0 ? 1 : 3;
        if ((i & 1) == 0) {
            const int f = nbr_cb(g, x, y, z, t, mu, dist);
            hop_load<NR, NT>(d, Uo[h] + mu * lstride, vhp, own_l, in,
                             (uint32_t)f * (uint32_t)sizeof(h16p), roff);
        } else {
            const int b = nbr_cb(g, x, y, z, t, mu, -dist);
            hop_load<NR, NT>(d, Ui[h] + mu * lstride, vhp, link_off<q16s>(b), in,
                             (uint32_t)b * (uint32_t)sizeof(h16p), roff);
        }
    };
#pragma unroll
    for (int i = 0; i < LA; ++i) load(i, buf[i]);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i + LA < 16) load(i + LA, buf[(i + LA) % (LA + 1)]);
        if ((i & 1) == 0) hop_math<NR, true>(buf[i % (LA + 1)], acc);
        else hop_math<NR, false>(buf[i % (LA + 1)], acc);
        hop_fence<NR>(acc);
    }
}

// roff[r]: byte offset of the lane's r-th RHS plane from the group's first
// (clamped to its last valid RHS in a ragged group, so that no lane branches).
template <int NR, bool NT, typename R, typename VS, typename LS>
__device__ __forceinline__ void hop_forward(const LS *__restrict__ U, int vh, uint32_t uoff,
                                            const VS *__restrict__ in, uint32_t voff,
                                            const uint32_t (&roff)[NR], vec2<R> (&acc)[NR][3]) {
    using V = vec2<R>;
    V u[9];
    const gptr<const LS> up = at(U, uoff);
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = Conv<LS>::template ld<R>(ldlink<NT>(up + k * kLinkTile));
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        {
            const V v0 = Conv<VS>::template ld<R>(*at(in, roff[r] + voff));
            const V v1 = Conv<VS>::template ld<R>(*at(in + vh, roff[r] + voff));
            const V v2 = Conv<VS>::template ld<R>(*at(in + 2 * (int64_t)vh, roff[r] + voff));
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
    hop_fence<NR>(acc);
}

// acc -= U^H v, with U read at the neighbour's index (offset noff for both).
template <int NR, bool NT, typename R, typename VS, typename LS>
__device__ __forceinline__ void hop_backward(const LS *__restrict__ U, int vh, uint32_t uoff,
                                             const VS *__restrict__ in, uint32_t voff,
                                             const uint32_t (&roff)[NR], vec2<R> (&acc)[NR][3]) {
    using V = vec2<R>;
    V u[9];
    const gptr<const LS> up = at(U, uoff);
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = Conv<LS>::template ld<R>(ldlink<NT>(up + k * kLinkTile));
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        {
            const V v0 = Conv<VS>::template ld<R>(*at(in, roff[r] + voff));
            const V v1 = Conv<VS>::template ld<R>(*at(in + vh, roff[r] + voff));
            const V v2 = Conv<VS>::template ld<R>(*at(in + 2 * (int64_t)vh, roff[r] + voff));
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
    hop_fence<NR>(acc);
}

// The generic hops split into loads and arithmetic (the arithmetic of
// hop_forward / hop_backward), for the pipelined loop below.
template <int NR, typename VS, typename LS>
struct HopRawG {
    LS u[9];
    VS v[NR][3];
};

template <int NR, bool NT, typename VS, typename LS>
__device__ __forceinline__ void hop_load_g(HopRawG<NR, VS, LS> &d, const LS *__restrict__ U,
                                           int vh, uint32_t uoff, const VS *__restrict__ in,
                                           uint32_t voff, const uint32_t (&roff)[NR]) {
    const gptr<const LS> up = at(U, uoff);
#pragma unroll
    for (int k = 0; k < 9; ++k) d.u[k] = ldlink<NT>(up + k * kLinkTile);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        d.v[r][0] = *at(in, roff[r] + voff);
        d.v[r][1] = *at(in + vh, roff[r] + voff);
        d.v[r][2] = *at(in + 2 * (int64_t)vh, roff[r] + voff);
    }
}

template <int NR, bool FWD, typename R, typename VS, typename LS>
__device__ __forceinline__ void hop_math_g(const HopRawG<NR, VS, LS> &d, vec2<R> (&acc)[NR][3]) {
    using V = vec2<R>;
    V u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = Conv<LS>::template ld<R>(d.u[k]);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const V v0 = Conv<VS>::template ld<R>(d.v[r][0]);
        const V v1 = Conv<VS>::template ld<R>(d.v[r][1]);
        const V v2 = Conv<VS>::template ld<R>(d.v[r][2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            V s = acc[r][a];
            if constexpr (FWD) {
                s.x = fma(u[3 * a].x, v0.x, s.x);  s.x = fma(-u[3 * a].y, v0.y, s.x);
                s.y = fma(u[3 * a].x, v0.y, s.y);  s.y = fma(u[3 * a].y, v0.x, s.y);
                s.x = fma(u[3 * a + 1].x, v1.x, s.x);  s.x = fma(-u[3 * a + 1].y, v1.y, s.x);
                s.y = fma(u[3 * a + 1].x, v1.y, s.y);  s.y = fma(u[3 * a + 1].y, v1.x, s.y);
                s.x = fma(u[3 * a + 2].x, v2.x, s.x);  s.x = fma(-u[3 * a + 2].y, v2.y, s.x);
                s.y = fma(u[3 * a + 2].x, v2.y, s.y);  s.y = fma(u[3 * a + 2].y, v2.x, s.y);
            } else {
                s.x = fma(-u[a].x, v0.x, s.x);  s.x = fma(-u[a].y, v0.y, s.x);
                s.y = fma(-u[a].x, v0.y, s.y);  s.y = fma(u[a].y, v0.x, s.y);
                s.x = fma(-u[3 + a].x, v1.x, s.x);  s.x = fma(-u[3 + a].y, v1.y, s.x);
                s.y = fma(-u[3 + a].x, v1.y, s.y);  s.y = fma(u[3 + a].y, v1.x, s.y);
                s.x = fma(-u[6 + a].x, v2.x, s.x);  s.x = fma(-u[6 + a].y, v2.y, s.x);
                s.y = fma(-u[6 + a].x, v2.y, s.y);  s.y = fma(u[6 + a].y, v2.x, s.y);
            }
            acc[r][a] = s;
        }
    }
}

// The 16 hops of a site in the order of the unpipelined loop, with the loads
// of hop i + LA issued before the arithmetic of hop i.
template <int NR, int LA, bool NT, typename R, typename VS, typename LS>
__device__ __forceinline__ void gen_hops_all(const LS *const (&Uo)[2], const LS *const (&Ui)[2],
                                             int64_t lstride, const Geom &g, int x, int y, int z,
                                             int t, uint32_t own_l, const VS *__restrict__ in,
                                             const uint32_t (&roff)[NR],
                                             vec2<R> (&acc)[NR][3]) {
    HopRawG<NR, VS, LS> buf[LA + 1];
    auto load = [&](int i, HopRawG<NR, VS, LS> &d) {
        const int h = i >> 3, mu = (i >> 1) & 3;
        const int dist = h == 0 ? 1 : 3;
        if ((i & 1) == 0) {
            const int f = nbr_cb(g, x, y, z, t, mu, dist);
            hop_load_g<NR, NT>(d, Uo[h] + mu * lstride, g.vh, own_l, in,
                               (uint32_t)f * (uint32_t)sizeof(VS), roff);
        } else {
            const int b = nbr_cb(g, x, y, z, t, mu, -dist);
            hop_load_g<NR, NT>(d, Ui[h] + mu * lstride, g.vh, link_off<LS>(b), in,
                               (uint32_t)b * (uint32_t)sizeof(VS), roff);
        }
    };
#pragma unroll
    for (int i = 0; i < LA; ++i) load(i, buf[i]);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i + LA < 16) load(i + LA, buf[(i + LA) % (LA + 1)]);
        if ((i & 1) == 0) hop_math_g<NR, true, R>(buf[i % (LA + 1)], acc);
        else hop_math_g<NR, false, R>(buf[i % (LA + 1)], acc);
        hop_fence<NR>(acc);
    }
}

// Epilogue of one RHS at one site for packed 16-bit vectors: o = cd acc
// (+ ca aux), rounded to 16 bits against the largest |component| of the
// three colours, stored with that norm; with DOT, dot += Re<aux, o> of the
// stored (rounded) o.  aux/out: the RHS's field, off: the site's byte offset.
template <bool AUX, bool DOT>
__device__ __forceinline__ void h16_epilogue(const vec2<float> (&acc)[3], float cd, float ca,
                                             const h16p *aux, h16p *out, uint32_t off,
                                             double &dot) {
    vec2<float> o[3], ax[3];
    if constexpr (AUX) {
        h16c c[3];
        float n;
        h16_unpack(__builtin_nontemporal_load(at(aux, off)), c, n);
        const float sc = n * (1.0f / kQ16);
#pragma unroll
        for (int k = 0; k < 3; ++k) ax[k] = vec2<float>{(float)c[k].x * sc, (float)c[k].y * sc};
    }
    float m = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o[k] = acc[k] * cd;
        if constexpr (AUX) {
            o[k].x = fmaf(ca, ax[k].x, o[k].x);
            o[k].y = fmaf(ca, ax[k].y, o[k].y);
        }
        m = fmaxf(m, fmaxf(fabsf(o[k].x), fabsf(o[k].y)));
    }
    const float qs = m > 0.0f ? kQ16 / m : 0.0f, ds = m * (1.0f / kQ16);
    h16c qv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        qv[k] = h16c{(short)rintf(o[k].x * qs), (short)rintf(o[k].y * qs)};
        if constexpr (AUX && DOT)  // the partial of the stored (rounded) output
            dot = fma((double)ax[k].x, (double)(qv[k].x * ds),
                      fma((double)ax[k].y, (double)(qv[k].y * ds), dot));
    }
    // the epilogue field and the output are touched once per launch: streamed
    // past L2, which keeps its lines for the neighbour gathers (48^3 x 96, 12
    // RHS: 1716/1877 -> 1690/1860 us)
    __builtin_nontemporal_store(h16p{__builtin_bit_cast(int, qv[0]), __builtin_bit_cast(int, qv[1]),
                                     __builtin_bit_cast(int, qv[2]), __float_as_int(m)},
                                at(out, off));
}

// Sum of x[0 .. kSites) in the canonical order, by one full wave (result in
// every lane): lane l adds x[l], x[l+64], x[l+128], x[l+192] in that order,
// then the fixed butterfly over the wave.
__device__ __forceinline__ double chunk_sum(const double *x) {
    static_assert(kSites == 4 * kWave, "canonical chunk is four waves of sites");
    const int l = threadIdx.x & (kWave - 1);
    double v = x[l];
    v += x[l + kWave];
    v += x[l + 2 * kWave];
    v += x[l + 3 * kWave];
    return wave_sum(v);
}

template <typename R, typename VS, typename LS, int NR, int LPS, bool AUX, bool AUX2, bool DOT,
          bool NT>
__global__ __launch_bounds__(kSites *LPS) void k_dslash(DslashArgs<R, VS, LS> a) {
    using V = vec2<R>;
    constexpr int SPW = kWave / LPS;  // sites per wave
    constexpr int RG = LPS * NR;      // RHS per group
    const Geom g = a.geom;
    const int vh = g.vh;
    const int lb = remap_block(a.xcd_remap, (int)blockIdx.x, (int)gridDim.x);
    int sb, grp;
    if (a.group_outer) {
        grp = lb / a.nsb;
        sb = lb - grp * a.nsb;
    } else {
        sb = lb / a.ngroups;
        grp = lb - sb * a.ngroups;
    }
    const int w = threadIdx.x / kWave, l = threadIdx.x & (kWave - 1);
    const int q = l / SPW;                    // RHS slot of this lane
    const int sl = w * SPW + (l - q * SPW);   // site within the block
    const int cb = sb * kSites + sl;
    const int rg0 = grp * RG;                 // first RHS of the group
    const int nr = min(NR, a.nrhs - rg0 - q * NR);
    // byte offset of this lane's first RHS plane within the group
    constexpr int CP = planes<VS>();
    const uint32_t qoff = (uint32_t)(q * NR * CP) * (uint32_t)vh * (uint32_t)sizeof(VS);

    double dotv[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) dotv[r] = 0.0;

    if (a.rhs_status) {
        // skip a group whose right-hand sides no longer iterate (block-uniform)
        bool any = false;
        for (int j = rg0; j < min(rg0 + RG, a.nrhs); ++j) any = any || a.rhs_status[j] == CG_ACTIVE;
        if (!any) {
            if (DOT && threadIdx.x < RG && rg0 + (int)threadIdx.x < a.nrhs)
                a.partials[(int64_t)(rg0 + threadIdx.x) * a.nsb + sb] = 0.0;
            return;
        }
    }

    if (cb < vh && nr > 0) {
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

        const VS *in = a.in + (int64_t)rg0 * CP * vh;
        uint32_t roff[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r)
            roff[r] = qoff + (uint32_t)(CP * min(r, nr - 1)) * (uint32_t)vh * (uint32_t)sizeof(VS);
        const int64_t lstride = 9 * kLinkTile * link_tiles(vh);  // one direction
        const uint32_t own = (uint32_t)cb * (uint32_t)sizeof(VS);
        const uint32_t own_l = link_off<LS>(cb);

        static_assert(!is_normed<VS>() || int_hops<VS, LS>(),
                      "packed 16-bit vectors are read with q16s links only");
        if constexpr (int_hops<VS, LS>()) {
            const q16s *const Uo[2] = {a.fat_out, a.lng_out};
            const q16s *const Ui[2] = {a.fat_in, a.lng_in};
            int_hops_all<NR, int_lookahead(NR, LPS), NT>(Uo, Ui, lstride, g, x, y, z, t, own_l, in,
                                                         roff, acc);
        } else if constexpr (gen_lookahead(NR, LPS, sizeof(R), sizeof(VS), sizeof(LS), false) > 0) {
            const LS *const Uo[2] = {a.fat_out, a.lng_out};
            const LS *const Ui[2] = {a.fat_in, a.lng_in};
            gen_hops_all<NR, gen_lookahead(NR, LPS, sizeof(R), sizeof(VS), sizeof(LS), false), NT,
                         R>(Uo, Ui, lstride, g, x, y, z, t, own_l, in, roff, acc);
        } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int hop = h == 0 ? 1 : 3;
            const LS *Uo = h == 0 ? a.fat_out : a.lng_out;
            const LS *Ui = h == 0 ? a.fat_in : a.lng_in;
            // mu = 0 (x)
            {
                const int f = (rowYZT * g.X + wrap(x + hop, g.X)) >> 1;
                const int b = (rowYZT * g.X + wrap(x - hop, g.X)) >> 1;
                const uint32_t bo = (uint32_t)b * (uint32_t)sizeof(VS);
                hop_forward<NR, NT, R>(Uo, vh, own_l, in, (uint32_t)f * (uint32_t)sizeof(VS), roff, acc);
                hop_backward<NR, NT, R>(Ui, vh, link_off<LS>(b), in, bo, roff, acc);
            }
            // mu = 1 (y)
            {
                const int f = ((((t * g.Z + z) * g.Y + wrap(y + hop, g.Y)) * g.X) + x) >> 1;
                const int b = ((((t * g.Z + z) * g.Y + wrap(y - hop, g.Y)) * g.X) + x) >> 1;
                const uint32_t bo = (uint32_t)b * (uint32_t)sizeof(VS);
                hop_forward<NR, NT, R>(Uo + lstride, vh, own_l, in, (uint32_t)f * (uint32_t)sizeof(VS), roff, acc);
                hop_backward<NR, NT, R>(Ui + lstride, vh, link_off<LS>(b), in, bo, roff, acc);
            }
            // mu = 2 (z)
            {
                const int f = ((((t * g.Z + wrap(z + hop, g.Z)) * g.Y + y) * g.X) + x) >> 1;
                const int b = ((((t * g.Z + wrap(z - hop, g.Z)) * g.Y + y) * g.X) + x) >> 1;
                const uint32_t bo = (uint32_t)b * (uint32_t)sizeof(VS);
                hop_forward<NR, NT, R>(Uo + 2 * lstride, vh, own_l, in, (uint32_t)f * (uint32_t)sizeof(VS), roff, acc);
                hop_backward<NR, NT, R>(Ui + 2 * lstride, vh, link_off<LS>(b), in, bo, roff, acc);
            }
            // mu = 3 (t)
            {
                const int f = ((((wrap(t + hop, g.T) * g.Z + z) * g.Y + y) * g.X) + x) >> 1;
                const int b = ((((wrap(t - hop, g.T) * g.Z + z) * g.Y + y) * g.X) + x) >> 1;
                const uint32_t bo = (uint32_t)b * (uint32_t)sizeof(VS);
                hop_forward<NR, NT, R>(Uo + 3 * lstride, vh, own_l, in, (uint32_t)f * (uint32_t)sizeof(VS), roff, acc);
                hop_backward<NR, NT, R>(Ui + 3 * lstride, vh, link_off<LS>(b), in, bo, roff, acc);
            }
        }
        }

        // epilogue
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
                for (int c = 0; c < 3; ++c) {
                    const int64_t plane = (int64_t)(rg0 * 3 + 3 * r + c) * vh;
                    const uint32_t off = qoff + own;
                    V o = acc[r][c] * a.cd;
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
        // per-block partial sums of Re<aux, out> for each RHS of the group, in
        // the canonical order over the block's sites; the CG update kernel adds
        // the blocks' partials in block order
        __shared__ double red[RG * kSites];
#pragma unroll
        for (int r = 0; r < NR; ++r) red[(q * NR + r) * kSites + sl] = dotv[r];
        __syncthreads();
        constexpr int NW = kSites * LPS / kWave;
        for (int j = w; j < RG; j += NW) {
            const double s = chunk_sum(red + j * kSites);
            if (l == 0 && rg0 + j < a.nrhs) a.partials[(int64_t)(rg0 + j) * a.nsb + sb] = s;
        }
    }
}

// Dynamic LDS a launch of kernel f requests (and leaves unused) so that at
// most `per_cu` of its blocks fit the 160 KiB of LDS of a compute unit; 0
// when per_cu is 0 (no cap).
inline size_t lds_cap_bytes(const void *f, int per_cu) {
    if (per_cu <= 0) return 0;
    hipFuncAttributes attr{};
    if (hipFuncGetAttributes(&attr, f) != hipSuccess) return 0;
    const size_t total = (size_t)kLdsPerCu / (size_t)per_cu / 512 * 512;
    return total > attr.sharedSizeBytes ? total - attr.sharedSizeBytes : 0;
}

template <typename R, typename VS, typename LS, int NR, int LPS, bool AUX, bool AUX2, bool DOT,
          bool NT>
void launch_one(const DslashArgs<R, VS, LS> &args, int nblocks, int per_cu, hipStream_t s) {
    auto *f = &k_dslash<R, VS, LS, NR, LPS, AUX, AUX2, DOT, NT>;
    // per cap, the LDS request + 1 once known (0: not yet asked)
    static std::atomic<int64_t> cache[kMaxBlocksPerCu + 1];
    const int k = per_cu < 0 ? 0 : (per_cu > kMaxBlocksPerCu ? kMaxBlocksPerCu : per_cu);
    int64_t v = cache[k].load(std::memory_order_relaxed);
    if (v == 0) {
        v = (int64_t)lds_cap_bytes(reinterpret_cast<const void *>(f), k) + 1;
        cache[k].store(v, std::memory_order_relaxed);
    }
    hipLaunchKernelGGL(f, dim3(nblocks), dim3(kSites * LPS), (size_t)(v - 1), s, args);
}

template <typename R, typename VS, typename LS, int NR, int LPS, bool NT>
void launch_variant(const DslashArgs<R, VS, LS> &args, int nblocks, bool aux, bool aux2, bool dot,
                    hipStream_t s) {
    const int cap = args.blocks_per_cu;
    if (dot)
        launch_one<R, VS, LS, NR, LPS, true, false, true, NT>(args, nblocks, cap, s);
    else if (aux2)
        launch_one<R, VS, LS, NR, LPS, true, true, false, NT>(args, nblocks, cap, s);
    else if (aux)
        launch_one<R, VS, LS, NR, LPS, true, false, false, NT>(args, nblocks, cap, s);
    else
        launch_one<R, VS, LS, NR, LPS, false, false, false, NT>(args, nblocks, cap, s);
}

template <typename R, typename VS, typename LS, int NR, int LPS>
hisq_status launch_shape(const DslashArgs<R, VS, LS> &args, int nblocks, bool aux, bool aux2,
                         bool dot, hipStream_t s) {
    if (args.ngroups == 1)
        launch_variant<R, VS, LS, NR, LPS, true>(args, nblocks, aux, aux2, dot, s);
    else
        launch_variant<R, VS, LS, NR, LPS, false>(args, nblocks, aux, aux2, dot, s);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

// True if the per-lane 32-bit byte offsets of the shape fit for this volume
// (site_bytes: bytes of one RHS's colour vector at one site: 48 FP64, 24
// FP32, 12 BF16, 16 packed 16-bit).
inline bool shape_fits(int nr, int lps, int vh, size_t site_bytes) {
    const uint64_t span = (uint64_t)(lps * nr) * (uint64_t)vh * site_bytes;
    return span < (1ull << 32);
}

// Storage kinds of the marching kernel: 0 FP64 vectors and links, 1 FP32
// vectors (FP32 or 16-bit links), 2 16-bit vectors and links; -1 none (BF16).
template <typename R, typename VS, typename LS>
constexpr int march_kind() {
    if constexpr (int_hops<VS, LS>()) return 2;
    else if constexpr (std::is_same<VS, vec2<double>>::value && std::is_same<LS, vec2<double>>::value)
        return 0;
    else if constexpr (std::is_same<VS, vec2<float>>::value &&
                       (std::is_same<LS, q16c>::value || std::is_same<LS, vec2<float>>::value))
        return 1;
    else return -1;
}

// (NR, LPS) shapes the marching kernel is built for, per storage kind.
__host__ __device__ constexpr bool march_shape_supported(int kind, int nr, int lps) {
    return kind == 2   ? (lps == 2 && (nr == 6 || nr == 3)) || (lps == 4 && nr == 3)
           : kind == 1 ? (lps == 2 && (nr == 6 || nr == 3)) || (lps == 4 && nr == 3)
           : kind == 0 ? lps == 2 && (nr == 1 || nr == 2 || nr == 3)
                       : false;
}

// The marching kernel (dslash_march.h), instantiated in dslash_march_*.hip
// for the storage kinds and shapes march_shape_supported() lists.
template <typename R, typename VS, typename LS>
hisq_status launch_march(const DslashArgs<R, VS, LS> &a, const DslashShape &sh, bool aux,
                         bool aux2, bool dot, hipStream_t s);

// Fill the argument block and launch with the given shape.
template <typename R, typename VS = vec2<R>, typename LS = vec2<R>>
hisq_status launch_dslash_t(const Geom &geom, const LS *const fat[2], const LS *const lng[2],
                            int out_parity, const VS *in, VS *out, int nrhs, const VS *aux,
                            double ca, const VS *aux2, double cb, double cd, double *partials,
                            DslashShape sh, hipStream_t s, const double *ca_rhs = nullptr,
                            const int *rhs_status = nullptr) {
    if (aux2 && !aux) return fail(HISQ_ERR_INVALID_ARG, "dslash: aux2 needs aux");
    if (is_normed<VS>() && aux2)
        return fail(HISQ_ERR_INVALID_ARG, "dslash: no second epilogue field for 16-bit vectors");
    if (!shape_fits(sh.nr, sh.lps, geom.vh, planes<VS>() * sizeof(VS)))
        return fail(HISQ_ERR_INVALID_ARG, "dslash: RHS group too large for this volume");
    DslashArgs<R, VS, LS> a{};
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
    a.ca_rhs = ca_rhs;
    a.rhs_status = rhs_status;
    a.geom = geom;
    a.out_parity = p;
    a.xcd_remap = sh.xcd_remap;
    a.group_outer = sh.group_outer;
    a.blocks_per_cu = sh.blocks_per_cu;
    a.nrhs = nrhs;
    a.ngroups = (nrhs + sh.lps * sh.nr - 1) / (sh.lps * sh.nr);
    a.nsb = (geom.vh + kSites - 1) / kSites;
    a.partials = partials;
    const bool dot = partials != nullptr;
    const int nblocks = a.nsb * a.ngroups;
    const bool x = aux != nullptr, x2 = aux2 != nullptr;
    if constexpr (march_kind<R, VS, LS>() >= 0)
        if (sh.march > 0) return launch_march<R, VS, LS>(a, sh, x, x2, dot, s);
#define HISQ_SHAPE(NR_, LPS_)                                                            \
    if (sh.nr == NR_ && sh.lps == LPS_)                                                  \
    return launch_shape<R, VS, LS, NR_, LPS_>(a, nblocks, x, x2, dot, s)
    HISQ_SHAPE(1, 1);
    HISQ_SHAPE(2, 1);
    HISQ_SHAPE(3, 1);
    HISQ_SHAPE(4, 1);
    HISQ_SHAPE(6, 1);
    HISQ_SHAPE(12, 1);
    HISQ_SHAPE(1, 2);
    HISQ_SHAPE(3, 2);
    HISQ_SHAPE(6, 2);
    HISQ_SHAPE(1, 4);
    HISQ_SHAPE(3, 4);
    HISQ_SHAPE(6, 4);
#undef HISQ_SHAPE
    return fail(HISQ_ERR_INVALID_ARG, "dslash: unsupported launch shape");
}

}  // namespace dslash_impl
}  // namespace hisq
