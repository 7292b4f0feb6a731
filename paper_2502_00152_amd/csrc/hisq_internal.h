// Internal declarations shared by the libhisq translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstdint>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hisq.h"

namespace hisq {

// ------------------------------------------------------------------ errors
struct Error {
    hisq_status status;
    std::string msg;
};

void set_error(const std::string &msg);
hisq_status fail(hisq_status st, const std::string &msg);

#define HISQ_HIP(call)                                                             \
    do {                                                                           \
        hipError_t hisq_he_ = (call);                                              \
        if (hisq_he_ != hipSuccess)                                                \
            return ::hisq::fail(hisq_he_ == hipErrorOutOfMemory ? HISQ_ERR_OOM : HISQ_ERR_HIP, \
                                std::string(#call) + ": " + hipGetErrorString(hisq_he_)); \
    } while (0)

#define HISQ_TRY(expr)                        \
    do {                                      \
        hisq_status hisq_st_ = (expr);        \
        if (hisq_st_ != HISQ_OK) return hisq_st_; \
    } while (0)

// --------------------------------------------------------------- geometry
// Lattice extents and derived sizes, passed by value to kernels.
struct Geom {
    int X, Y, Z, T;
    int Xh;        // X / 2
    int vh;        // X*Y*Z*T / 2
};

// ------------------------------------------------------------- workspace
// Device scratch buffers owned by a gauge handle, grown on demand and kept
// until the handle is destroyed.
class Workspace {
public:
    ~Workspace();
    hisq_status get(const char *name, size_t bytes, void **ptr);
    void release();
    // free one named buffer (after its last use has completed)
    void release_one(const char *name);

private:
    struct Buf {
        void *ptr = nullptr;
        size_t bytes = 0;
    };
    std::map<std::string, Buf> bufs_;
};

}  // namespace hisq

namespace hisq {
// Link storage is tiled by kLinkTile consecutive checkerboard sites: within a
// tile the 9 entries of the colour matrix are kLinkTile apart, so a wave reads
// entry k of its sites at a constant offset from entry 0.
constexpr int kLinkTile = 16;
__host__ __device__ inline int64_t link_tiles(int vh) { return (vh + kLinkTile - 1) / kLinkTile; }
// complex entries per parity array (4 directions, padded to whole tiles)
inline int64_t link_array_entries(int vh) { return 4 * 9 * kLinkTile * link_tiles(vh); }
__host__ __device__ inline int64_t link_index(int mu, int k, int cb, int64_t ntiles) {
    return (((int64_t)mu * ntiles + (cb / kLinkTile)) * 9 + k) * kLinkTile + (cb % kLinkTile);
}
}  // namespace hisq

// The gauge handle: links in kernel layout plus scratch.
//   fat[p], lng[p]: links living on sites of parity p, complex, entry k of the
//   3x3 row-major matrix of direction mu at checkerboard site cb is at
//   link_index(mu, k, cb, link_tiles(Vh)): [4 mu][tile][9 k][kLinkTile].
struct hisq_gauge_s {
    hisq::Geom geom;
    int device = 0;
    double2 *fat[2] = {nullptr, nullptr};
    double2 *lng[2] = {nullptr, nullptr};
    float2 *fat32[2] = {nullptr, nullptr};  // FP32 copies, made on first sloppy use
    float2 *lng32[2] = {nullptr, nullptr};
    uint32_t *fat16[2] = {nullptr, nullptr}; // BF16 copies (two bfloat16 per complex),
    uint32_t *lng16[2] = {nullptr, nullptr}; //   made on first BF16 use
    int32_t *fatq[2] = {nullptr, nullptr};   // 16-bit fixed-point copies (two int16
    int32_t *lngq[2] = {nullptr, nullptr};   //   per complex), made on first use,
    double q16_step = 0.0;                   //   value = integer * q16_step
    int32_t *fatn[2] = {nullptr, nullptr};   // the same with components in
    int32_t *lngn[2] = {nullptr, nullptr};   //   [-qn_max, qn_max] (integer-dot
    double qn_step = 0.0;                    //   stencil; q16s layout of
                                             //   dslash_kernel.h), value = integer * qn_step
    int qn_max = 0;                          //   largest integer component of that copy
    double link_absmax = -1.0;               // largest |component| of fat and long
    hipStream_t cg_stream = nullptr;        // the solvers' own stream (capturable)
    hisq::Workspace ws;
};

namespace hisq {

// ------------------------------------------------------------ profiling
// While an object of this class lives, ProfileScope records nothing on the
// calling thread (the allocation-free entry points create no events).
class ProfileSuppress {
public:
    ProfileSuppress();
    ~ProfileSuppress();

private:
    bool prev_;
};

// Event-timed launches, per kernel class.
class ProfileScope {
public:
    ProfileScope(const char *cls, hipStream_t s);
    ~ProfileScope();

private:
    int slot_ = -1;
    hipStream_t s_;
    const char *cls_;
};

// ------------------------------------------------- CG per-RHS device state
enum CgStatus : int {
    CG_ACTIVE = 0,
    CG_PENDING = 1,     // iterated residual passed: waits for a true-residual check
    CG_CONVERGED = 2,
    CG_RESTART = 3,     // true residual failed: p must be rebuilt from the true r
    CG_MAXITER = 4,
    CG_BREAKDOWN = 5,
    CG_NAN = 6,
};

// Arrays of nrhs entries each, in device memory.
struct CgDev {
    double *rho;       // <r, r> of the current residual
    double *rho_pend;  // iterated <r, r> that triggered a pending check
    double *alpha;
    double *beta;
    double *bnorm2;
    double *tol2b;     // tol^2 ||b||^2
    double *true_res2; // last true ||b - A x||^2
    int *status;
    int *iters;
    int *checks;
    double *xp_alpha;  // the x/p update of this iteration: x += xp_alpha p,
    double *xp_beta;   //   p = r + xp_beta p
    int *xp_mode;      // 0: none, 1: x only, 2: x and p
    double *rho_ru;    // mixed precision: true ||r||^2 at the last reliable update
    int *ru_flag;      // mixed precision: set when a reliable update is due
    double delta2;     // mixed precision: reliable_delta^2 (0: no delta trigger)
    int ru_freeze;     // mixed precision: 1 = a delta trigger stops the RHS's
                       // recurrence until the reliable update (0: it goes on
                       // until the host's next poll)
    int max_iter;
};

// Per-block partial sums of a reduction, [nvals][nblocks]; every launch writes
// all of its entries before a later kernel adds them in block order.
// hisq_set_tuning "cg_reliable_freeze" (-1 automatic, 0, 1)
extern int64_t g_ru_freeze;

struct Reduce {
    double *partials;
};

// ------------------------------------------------------- kernel launchers
enum DslashFinal : int {
    FIN_NONE = 0,
    FIN_CG_ALPHA = 1,   // store per-block partial sums of Re<aux, out> per RHS
};

// out = ca * aux + cb * aux2 + cd * D_{p,1-p} in.  aux/aux2 may be null (their
// coefficient is then ignored; aux2 needs aux); aux and aux2 may alias out.
// ca_rhs (device, nrhs doubles), if set, replaces ca by a value per RHS.
// With fin == FIN_CG_ALPHA, also stores per-block partials of Re<aux, out>
// in red->partials as [nrhs][dslash_reduce_blocks()].  With cg set, groups
// of RHS none of which is CG_ACTIVE are skipped (their output is left as is).
hisq_status launch_dslash(const hisq_gauge_s *g, int out_parity, const double2 *in,
                          double2 *out, int nrhs, const double2 *aux, double ca,
                          const double2 *aux2, double cb, double cd, DslashFinal fin,
                          const CgDev *cg, const Reduce *red, hipStream_t s,
                          const double *ca_rhs = nullptr);

// Launch-shape knobs of the half stencil (hisq_set_tuning).
hisq_status dslash_set_tuning(const std::string &key, int64_t value);

// Number of reduction blocks the dslash launch for (g, nrhs) uses.
int dslash_reduce_blocks(const hisq_gauge_s *g, int nrhs);

// BLAS for CG on parity vectors of n = 3*Vh complex entries per RHS.
int blas_reduce_blocks(int64_t n);
hisq_status cg_init(int64_t n, int nrhs, const double2 *b, const double2 *Ax, double2 *r,
                    double2 *p, double tol, const CgDev &cg, const Reduce &red,
                    hipStream_t s);
// alpha from the <p, Ap> partials (pap, nb_pap per RHS); r -= alpha Ap with
// partials of ||r||^2 into red; cg_finalize advances the per-RHS state;
// cg_update_xp then does x += alpha p and p = r + beta p (old p in both).
hisq_status cg_update_r(int64_t n, int nrhs, double2 *r, const double2 *Ap, const double *pap,
                        int nb_pap, const CgDev &cg, const Reduce &red, hipStream_t s);
// From kPapPresum stencil blocks per RHS up, the CG sums the <p, A p>
// partials once per iteration (cg_sum_pap: pq[j], a block per RHS, in one
// fixed order) and the r update and the state kernel read that one value per
// RHS, instead of every r-update block re-reading all partials (at 48^3 x 96,
// 20736 per RHS); below it they sum the partials themselves.
constexpr int kPapPresum = 1024;
hisq_status cg_sum_pap(int nrhs, const double *pap, int nb_pap, double *pq, hipStream_t s);
hisq_status cg_finalize(int64_t n, int nrhs, const double *pap, int nb_pap, const CgDev &cg,
                        const Reduce &red, hipStream_t s);
hisq_status cg_update_xp(int64_t n, int nrhs, double2 *x, const double2 *r, double2 *p,
                         const CgDev &cg, hipStream_t s);
// FP32 (sloppy) versions: FP32 vectors, FP64 scalars and reductions.
hisq_status cg_update_r(int64_t n, int nrhs, float2 *r, const float2 *Ap, const double *pap,
                        int nb_pap, const CgDev &cg, const Reduce &red, hipStream_t s);
hisq_status cg_update_xp(int64_t n, int nrhs, float2 *x, const float2 *r, float2 *p,
                         const CgDev &cg, hipStream_t s);
hisq_status cg_true_residual(int64_t n, int nrhs, const double2 *b, const double2 *Ax,
                             double2 *r, const CgDev &cg, const Reduce &red, bool final_only,
                             hipStream_t s);
hisq_status cg_restart_p(int64_t n, int nrhs, const double2 *r, double2 *p, const CgDev &cg,
                         hipStream_t s);

// Layout conversion.
hisq_status launch_split(const hisq_gauge_s *g, const double2 *full, double2 *even,
                         double2 *odd, int nrhs, hipStream_t s);
hisq_status launch_merge(const hisq_gauge_s *g, const double2 *even, const double2 *odd,
                         double2 *full, int nrhs, hipStream_t s);
hisq_status launch_pack_links(const hisq_gauge_s *g, const double2 *canon, double2 *soa[2],
                              double coef, unsigned flags, bool is_long, hipStream_t s);

// Complex tall-skinny contractions on the FP64 matrix cores (columns of N complex).
// C[j][i] = out_scale * row_scale[i] * sum_s conj(V[i][s]) B[j][s]   (C: [n][k] complex)
hisq_status gemm_tn(hisq_gauge_s *g, const double2 *V, int k, const double2 *B, int n,
                    int64_t N, const double *row_scale_dev, double out_scale, double2 *C,
                    hipStream_t s);
// X[j][s] = beta X[j][s] + sum_i V[i][s] C[j][i]
hisq_status gemm_nn(const double2 *V, int k, const double2 *C, int n, int64_t N, double beta,
                    double2 *X, hipStream_t s);
// The same with FP32 V (converted to FP64 on load; products and sums FP64).
hisq_status gemm_tn(hisq_gauge_s *g, const float2 *V, int k, const double2 *B, int n,
                    int64_t N, const double *row_scale_dev, double out_scale, double2 *C,
                    hipStream_t s);
hisq_status gemm_nn(const float2 *V, int k, const double2 *C, int n, int64_t N, double beta,
                    double2 *X, hipStream_t s);
// The same over `rows` rows (a multiple of 8) of columns ldv and ldx complex
// numbers apart (a block of rows of larger matrices).
hisq_status gemm_nn_ld(const double2 *V, int64_t ldv, int k, const double2 *C, int n,
                       int64_t rows, double beta, double2 *X, int64_t ldx, hipStream_t s);

// FP32 (sloppy) half stencil; partials (optional) as for FIN_CG_ALPHA.
hisq_status ensure_links_f32(hisq_gauge_s *g, hipStream_t s);
hisq_status launch_dslash_f32(hisq_gauge_s *g, int out_parity, const float2 *in, float2 *out,
                              int nrhs, const float2 *aux, double ca, const float2 *aux2, double cb,
                              double cd, double *partials, hipStream_t s,
                              const double *ca_rhs = nullptr, const int *rhs_status = nullptr);
hisq_status apply_mdagm_f32(hisq_gauge_s *g, double two_m, const float2 *in, float2 *out, int nrhs,
                            double *partials, hipStream_t s);

// BF16 storage (uint32_t = two bfloat16: real part low, imaginary part high).
hisq_status ensure_links_bf16(hisq_gauge_s *g, hipStream_t s);
// FP64 -> BF16, rounded to nearest even (n complex numbers)
hisq_status convert_double_to_bf16(const double2 *src, uint32_t *dst, int64_t n, hipStream_t s);
// half stencil with BF16 vectors and links (FP32 arithmetic)
hisq_status launch_dslash_bf16(hisq_gauge_s *g, int out_parity, const uint32_t *in, uint32_t *out,
                               int nrhs, const uint32_t *aux, double ca, const uint32_t *aux2,
                               double cb, double cd, hipStream_t s);
hisq_status apply_mdagm_bf16(hisq_gauge_s *g, double two_m, const uint32_t *in, uint32_t *out,
                             int nrhs, hipStream_t s);
// half stencil with FP32 vectors and BF16 links: the sloppy operator at
// sloppy_prec = HISQ_BF16 (arguments as launch_dslash_f32, without aux2)
hisq_status launch_dslash_f32_bl(hisq_gauge_s *g, int out_parity, const float2 *in, float2 *out,
                                 int nrhs, const float2 *aux, double ca, double cd,
                                 double *partials, hipStream_t s, const double *ca_rhs = nullptr,
                                 const int *rhs_status = nullptr);
// 16-bit fixed-point links (HISQ_Q16): FP32 vectors and arithmetic
hisq_status ensure_links_q16(hisq_gauge_s *g, hipStream_t s);
// the copy with components in [-kQLinkNarrow, kQLinkNarrow] read by the
// stencil on 16-bit vectors
hisq_status ensure_links_q16n(hisq_gauge_s *g, hipStream_t s);
hisq_status launch_dslash_f32_q16(hisq_gauge_s *g, int out_parity, const float2 *in, float2 *out,
                                  int nrhs, const float2 *aux, double ca, double cd,
                                  double *partials, hipStream_t s, const double *ca_rhs = nullptr,
                                  const int *rhs_status = nullptr);
hisq_status apply_mdagm_q16(hisq_gauge_s *g, double two_m, const float2 *in, float2 *out, int nrhs,
                            hipStream_t s);
// 16-bit fixed-point vector fields (HISQ_HALF): [nrhs][3][Vh] int16 pairs, then
// [nrhs][Vh] float norms (the largest |component| of the site); the stencil
// with 16-bit links, and the CG updates on such p and A p
int64_t half_field_bytes(int64_t vh, int nrhs);
hisq_status launch_dslash_h16(hisq_gauge_s *g, int out_parity, const void *in, void *out,
                              int nrhs, const void *aux, double ca, double cd, double *partials,
                              hipStream_t s, const double *ca_rhs = nullptr,
                              const int *rhs_status = nullptr);
hisq_status half_update_r(int64_t vh, int nrhs, float2 *r, const void *ap, const double *pap,
                          int nb_pap, const CgDev &cg, const Reduce &red, hipStream_t s);
hisq_status half_update_xp(int64_t vh, int nrhs, float2 *x, const float2 *r, void *p,
                           const CgDev &cg, hipStream_t s);
// p = r + beta p (mode 1) or p = r (mode 2) per RHS; mode null: p = r for all
hisq_status half_p_restart(int64_t vh, int nrhs, void *p, const float2 *r, const double *beta,
                           const int *mode, hipStream_t s);
hisq_status half_to_f32(int64_t vh, int nrhs, const void *h, float2 *out, hipStream_t s);
// the operators at HISQ_HALF (FP32 vectors at the boundary, 16-bit inside)
hisq_status apply_dslash_half(hisq_gauge_s *g, int out_parity, const float2 *in, float2 *out,
                              int nrhs, hipStream_t s);
hisq_status apply_mdagm_half(hisq_gauge_s *g, double two_m, const float2 *in, float2 *out,
                             int nrhs, hipStream_t s);

// The CG drivers run on the handle's own non-blocking stream (created on first
// use, default priority), ordered after the caller's stream on entry and
// before it on exit.  Chunks of iterations can then be captured into a HIP
// graph and replayed (one launch instead of five per iteration).
hisq_status solver_stream(hisq_gauge_s *g, hipStream_t caller, hipStream_t *out);
hisq_status solver_stream_done(hisq_gauge_s *g, hipStream_t caller);
// True if the iteration chunks of a solve of nrhs RHS should be graph-captured.
bool cg_use_graphs(const hisq_gauge_s *g, int nrhs);

// A captured chunk of iterations, replayed with one launch.
class GraphChunk {
public:
    ~GraphChunk();
    // Capture `body` (stream-ordered launches on s, nothing else) on first use,
    // then launch the instantiated graph.
    template <typename F>
    hisq_status run(hipStream_t s, F &&body) {
        if (!exec_) {
            HISQ_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            const hisq_status st = body();
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &graph);
            if (st != HISQ_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            HISQ_HIP(e);
            graph_ = graph;
            HISQ_HIP(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
        }
        HISQ_HIP(hipGraphLaunch(exec_, s));
        return HISQ_OK;
    }

private:
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
};

// Chunks of CG iterations of several systems, one host thread each,
// launched as one HIP graph (hisq_cg_solve_multi with "cg_multi_graph").
// Each solver hands its chunk (stream-ordered launches on its own stream) to
// the group and waits; the last member to arrive captures every member's
// chunk on the members' streams, forked from and joined to one origin
// stream, into one graph, launches it, and orders every member stream after
// it.  The instantiated graph is replayed while the members and their
// systems stay the same.  A member leaves when its thread has no system
// left.  Launch arguments of a chunk must not change between chunks of one
// system (the CG iteration kernels read all scalars from device memory).
class ChunkGroup {
public:
    explicit ChunkGroup(int members) : active_(members) {}
    ~ChunkGroup();
    // member `sys` (a system index) runs `body` on stream s as part of the
    // next combined launch
    hisq_status run(hipStream_t s, int sys, const std::function<hisq_status()> &body);
    void leave();

private:
    struct Pending {
        hipStream_t s;
        int sys;
        const std::function<hisq_status()> *body;
    };
    void launch_locked();
    hisq_status capture_locked();
    std::mutex mu_;
    std::condition_variable cv_;
    int active_;
    uint64_t round_ = 0;
    hisq_status round_status_ = HISQ_OK;
    std::string round_error_;
    std::vector<Pending> pending_;
    std::vector<std::pair<hipStream_t, int>> key_;  // members of the cached graph
    hipStream_t origin_ = nullptr;
    std::vector<hipEvent_t> events_;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
};
// hisq_set_tuning "cg_multi_graph" is 1 (and kernel timing is off)
bool cg_multi_graph();
// the group this thread's CG solves hand their chunks to (null: none), and
// the index of the system being solved
extern thread_local ChunkGroup *t_chunk_group;
extern thread_local int t_chunk_sys;

// Mixed-precision CG helpers; mask (nrhs ints, device) selects RHS, null = all.
hisq_status mixed_to_f32(const double2 *src, float2 *dst, int64_t n, int nrhs, const int *mask,
                         hipStream_t s);
// x += xs; xs = 0
hisq_status mixed_accum_x(double2 *x, float2 *xs, int64_t n, int nrhs, const int *mask,
                          hipStream_t s);
// r = b - Ax and out[j] = ||r_j||^2 (0 for unmasked RHS), partials in red as
// [nrhs][mixed_resid_blocks(n)]
hisq_status mixed_resid(const double2 *b, const double2 *Ax, double2 *r, int64_t n, int nrhs,
                        const int *mask, double *out, const Reduce &red, hipStream_t s);
int mixed_resid_blocks(int64_t n);
// per RHS by mode[j]: 0 keep p, 1 p = r + beta[j] p, 2 p = r
hisq_status mixed_p_restart(float2 *p, const float2 *r, int64_t n, int nrhs, const double *beta,
                            const int *mode, hipStream_t s);
// zero column j of C ([nrhs][k]) where mask[j] == 0
hisq_status mixed_mask_rows(double2 *C, int k, int nrhs, const int *mask, hipStream_t s);
// Precision change of n complex numbers (FP64 <-> FP32, or a copy).
hisq_status convert_vectors(const void *src, hisq_prec sp, void *dst, hisq_prec dp, int64_t n,
                            hipStream_t s);
hisq_status solve_mixed(hisq_gauge_s *g, double two_m, const double2 *b, double2 *x, int nrhs,
                        const hisq_cg_params *P, hisq_cg_stats *stats, hipStream_t s,
                        const double *m2_rhs = nullptr, hisq_prec links = HISQ_FP32);

// Operators built from dslash.
// out = ((2m)^2 - D_{p,1-p} D_{1-p,p}) in on parity p (p = 0: the even operator A);
// m2_rhs (device, nrhs doubles), if set, gives (2m)^2 per RHS; skip (device,
// nrhs ints), if set, lets RHS groups whose entries are all nonzero be skipped
// (their output is left as is).
hisq_status apply_mdagm(hisq_gauge_s *g, double two_m, const double2 *in, double2 *out,
                        int nrhs, hipStream_t s, int parity = 0, const double *m2_rhs = nullptr,
                        const int *skip = nullptr);

}  // namespace hisq
