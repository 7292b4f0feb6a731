// Vector updates and FP64 global reductions of the CG iteration
// (arXiv:2502.00152, section 2: conjugate gradient on the even-odd
// preconditioned normal equation, stopped on the true residual).
//
// Each right-hand side r runs its own recurrence
//   alpha = rho / Re<p, Ap>;  x += alpha p;  r -= alpha Ap;
//   rho' = <r, r>;  beta = rho' / rho;  p = r + beta p
// The scalars live in device memory.  Reductions are deterministic: every
// block stores its partial sums and a later kernel adds them in block order.
// The per-iteration reductions avoid any cross-block synchronisation inside a
// kernel (a device-scope fence per block writes back L2 on this multi-XCD
// chip and costs more than the update itself): the r update re-sums the
// <p, Ap> partials of its own RHS in every block, a small kernel (one wave
// per RHS) advances the per-RHS state, and x and p are updated together
// afterwards (x += alpha p with the old p, then p = r + beta p).  The rare
// steps (initial and true residuals, restarts) work the same way: a pass
// that stores per-block partials, then a small kernel (one wave per RHS)
// that adds them in block order and takes the decision.  No kernel depends
// on a counter or on scratch memory being zero when it starts.
#include "device_util.h"
#include "hisq_internal.h"

namespace hisq {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int kBS = 256;

// Grid: x = blocks per RHS (grid-stride over n complex entries), y = RHS.
struct BlasGrid {
    int nbx;
    int64_t n;
};

BlasGrid make_grid(int64_t n) {
    BlasGrid g;
    g.n = n;
    int64_t nb = (n + 4 * kBS - 1) / (4 * kBS);
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    g.nbx = (int)nb;
    return g;
}

__device__ __forceinline__ double norm2(dvec2 v) { return fma(v.x, v.x, v.y * v.y); }

// r = b - Ax; p = r; partials of ||b||^2 and ||r||^2 per RHS, stored as
// [2][nrhs][gridDim.x] (k_cg_init_state adds them).
__global__ __launch_bounds__(kBS) void k_cg_init(int64_t n, int nrhs, const dvec2 *__restrict__ b,
                                                 const dvec2 *__restrict__ Ax,
                                                 dvec2 *__restrict__ r, dvec2 *__restrict__ p,
                                                 double *__restrict__ partials) {
    const int rhs = blockIdx.y;
    const int64_t off = rhs * n;
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const dvec2 bb = b[off + i];
        const dvec2 rr = bb - Ax[off + i];
        r[off + i] = rr;
        p[off + i] = rr;
        v[0] += norm2(bb);
        v[1] += norm2(rr);
    }
    __shared__ double lds[2 * (kBS / kWave)];
    block_sum<2, kBS>(v, lds);
    const int nbx = gridDim.x;
    if (threadIdx.x == 0) {
        partials[(int64_t)rhs * nbx + blockIdx.x] = v[0];
        partials[(int64_t)(nrhs + rhs) * nbx + blockIdx.x] = v[1];
    }
}

// Fixed-order sum of nb partials by one wave (every caller gets the same bits):
// lane l adds partials l, l+64, ... in order, then a butterfly over the wave.
__device__ __forceinline__ double wave_sum_partials(const double *__restrict__ p, int nb) {
    const int lane = threadIdx.x & (kWave - 1);
    double v = 0.0;
    for (int i = lane; i < nb; i += kWave) v += p[i];
    return wave_sum(v);
}

// One wave per RHS: ||b||^2 and ||r||^2 from k_cg_init's partials, and the
// initial per-RHS state (every field the iteration reads is written here).
__global__ __launch_bounds__(kBS) void k_cg_init_state(int nrhs, const double *__restrict__ partials,
                                                       int nbx, double tol, CgDev cg) {
    const int q = blockIdx.x * (kBS / kWave) + threadIdx.x / kWave;
    if (q >= nrhs) return;
    const double bn = wave_sum_partials(partials + (int64_t)q * nbx, nbx);
    const double rn = wave_sum_partials(partials + (int64_t)(nrhs + q) * nbx, nbx);
    if ((threadIdx.x & (kWave - 1)) != 0) return;
    cg.bnorm2[q] = bn;
    cg.tol2b[q] = tol * tol * bn;
    cg.rho[q] = rn;
    cg.rho_pend[q] = rn;
    cg.true_res2[q] = rn;
    cg.iters[q] = 0;
    cg.checks[q] = 0;
    cg.alpha[q] = 0.0;
    cg.beta[q] = 0.0;
    cg.xp_alpha[q] = 0.0;
    cg.xp_beta[q] = 0.0;
    cg.xp_mode[q] = 0;
    if (!isfinite(bn) || !isfinite(rn))
        cg.status[q] = CG_NAN;
    else if (bn == 0.0 || rn <= tol * tol * bn)
        cg.status[q] = CG_CONVERGED;
    else
        cg.status[q] = CG_ACTIVE;
}

// alpha = rho / <p, Ap>, with <p, Ap> summed from the stencil kernel's
// per-block partials (every block repeats the same fixed-order sum);
// r -= alpha Ap and per-block partials of ||r||^2.
template <typename V>
__global__ __launch_bounds__(kBS) void k_cg_update_r(int64_t n, V *__restrict__ r,
                                                     const V *__restrict__ Ap,
                                                     const double *__restrict__ pap, int nb_pap,
                                                     CgDev cg, Reduce red) {
    using R = decltype(V{}.x);
    const int rhs = blockIdx.y;
    const int64_t off = rhs * n;
    __shared__ double pq_s;
    if (threadIdx.x < kWave) {
        const double v = wave_sum_partials(pap + (int64_t)rhs * nb_pap, nb_pap);
        if (threadIdx.x == 0) pq_s = v;
    }
    __syncthreads();
    const double pq = pq_s;
    double v[1] = {0.0};
    if (cg.status[rhs] == CG_ACTIVE && isfinite(pq) && pq > 0.0) {
        const R al = (R)(cg.rho[rhs] / pq);
        for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * kBS) {
            const V qq = Ap[off + i];
            V rr = r[off + i];
            rr.x = fma(-al, qq.x, rr.x);
            rr.y = fma(-al, qq.y, rr.y);
            r[off + i] = rr;
            v[0] += norm2(dvec2{(double)rr.x, (double)rr.y});
        }
    }
    __shared__ double lds[kBS / kWave];
    block_sum<1, kBS>(v, lds);
    if (threadIdx.x == 0) red.partials[(int64_t)rhs * gridDim.x + blockIdx.x] = v[0];
}

// pq[j] = RHS j's nb <p, A p> partials in one fixed order: one block of
// kSumBS threads per RHS, thread i adding entries i, i + kSumBS, ... in
// turn, then the block sum (waves in order).
constexpr int kSumBS = 1024;
__global__ __launch_bounds__(kSumBS) void k_sum_pap(const double *__restrict__ pap, int nb,
                                                    double *__restrict__ pq) {
    const int j = blockIdx.x;
    const double *p = pap + (int64_t)j * nb;
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nb; i += kSumBS) v[0] += p[i];
    __shared__ double lds[kSumBS / kWave];
    block_sum<1, kSumBS>(v, lds);
    if (threadIdx.x == 0) pq[j] = v[0];
}

// One wave per RHS: the per-RHS state machine after an r update.  x and p are
// updated afterwards by k_cg_update_xp with the alpha and beta written here.
__global__ __launch_bounds__(kBS) void k_cg_finalize(int nrhs, const double *__restrict__ pap,
                                                     int nb_pap, int nb_rr, CgDev cg,
                                                     Reduce red) {
    const int q = blockIdx.x * (kBS / kWave) + threadIdx.x / kWave;
    if (q >= nrhs) return;
    const double pq = wave_sum_partials(pap + (int64_t)q * nb_pap, nb_pap);
    const double rn = wave_sum_partials(red.partials + (int64_t)q * nb_rr, nb_rr);
    if ((threadIdx.x & (kWave - 1)) != 0) return;
    cg.xp_alpha[q] = 0.0;  // no x/p update unless the RHS was active in this iteration
    cg.xp_beta[q] = 0.0;
    cg.xp_mode[q] = 0;
    if (cg.status[q] != CG_ACTIVE) return;
    if (!isfinite(pq)) {
        cg.status[q] = CG_NAN;
        return;
    }
    if (!(pq > 0.0)) {
        cg.status[q] = CG_BREAKDOWN;
        return;
    }
    const double al = cg.rho[q] / pq;
    cg.alpha[q] = al;
    cg.xp_alpha[q] = al;
    cg.xp_mode[q] = 1;  // x += alpha p in any case (r already moved)
    cg.iters[q] += 1;
    if (!isfinite(rn)) {
        cg.status[q] = CG_NAN;
    } else if (rn <= cg.tol2b[q] ||
               (cg.ru_freeze && cg.delta2 > 0.0 && rn <= cg.delta2 * cg.rho_ru[q])) {
        // converged in the recurrence, or (ru_freeze) due for a reliable
        // update: the RHS waits for the host's FP64 true residual
        cg.rho_pend[q] = rn;
        cg.status[q] = CG_PENDING;
    } else {
        const double be = rn / cg.rho[q];
        cg.beta[q] = be;
        cg.rho[q] = rn;
        // mixed precision: the iterated residual fell by delta since the last
        // reliable update; the host runs it at its next poll (the recurrence
        // goes on meanwhile)
        if (cg.delta2 > 0.0 && rn <= cg.delta2 * cg.rho_ru[q]) cg.ru_flag[q] = 1;
        if (cg.iters[q] >= cg.max_iter) {
            cg.status[q] = CG_MAXITER;
        } else {
            cg.xp_beta[q] = be;
            cg.xp_mode[q] = 2;  // and p = r + beta p
        }
    }
}

// x += alpha p_old; p = r + beta p_old (mode 2), or only the x update (mode 1).
template <typename V>
__global__ __launch_bounds__(kBS) void k_cg_update_xp(int64_t n, V *__restrict__ x,
                                                      const V *__restrict__ r,
                                                      V *__restrict__ p, CgDev cg) {
    using R = decltype(V{}.x);
    const int rhs = blockIdx.y;
    const int mode = cg.xp_mode[rhs];
    if (mode == 0) return;
    const int64_t off = rhs * n;
    const R al = (R)cg.xp_alpha[rhs], be = (R)cg.xp_beta[rhs];
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const V pp = p[off + i];
        V xx = x[off + i];
        xx.x = fma(al, pp.x, xx.x);
        xx.y = fma(al, pp.y, xx.y);
        x[off + i] = xx;
        if (mode == 2) {
            const V rr = r[off + i];
            V np;
            np.x = fma(be, pp.x, rr.x);
            np.y = fma(be, pp.y, rr.y);
            p[off + i] = np;
        }
    }
}

// For pending RHS (or all, with final_only): r = b - Ax (stored unless
// final_only) and per-block partials of ||r||^2 (0 for the other RHS);
// k_cg_true_state takes the decisions.
__global__ __launch_bounds__(kBS) void k_cg_true_residual(int64_t n, const dvec2 *__restrict__ b,
                                                          const dvec2 *__restrict__ Ax,
                                                          dvec2 *__restrict__ r, CgDev cg,
                                                          double *__restrict__ partials,
                                                          int final_only) {
    const int rhs = blockIdx.y;
    const int64_t off = rhs * n;
    double v[1] = {0.0};
    if (final_only || cg.status[rhs] == CG_PENDING) {
        for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * kBS) {
            const dvec2 rr = b[off + i] - Ax[off + i];
            if (!final_only) r[off + i] = rr;
            v[0] += norm2(rr);
        }
    }
    __shared__ double lds[kBS / kWave];
    block_sum<1, kBS>(v, lds);
    if (threadIdx.x == 0) partials[(int64_t)rhs * gridDim.x + blockIdx.x] = v[0];
}

// One wave per RHS: the true ||r||^2 in block order; for a pending RHS the
// convergence decision (converged, out of iterations, or a restart of the
// recurrence from the true residual with beta = rho_true / rho).
__global__ __launch_bounds__(kBS) void k_cg_true_state(int nrhs, const double *__restrict__ partials,
                                                       int nbx, CgDev cg, int final_only) {
    const int q = blockIdx.x * (kBS / kWave) + threadIdx.x / kWave;
    if (q >= nrhs) return;
    const double tr = wave_sum_partials(partials + (int64_t)q * nbx, nbx);
    if ((threadIdx.x & (kWave - 1)) != 0) return;
    if (final_only) {
        cg.true_res2[q] = tr;
        return;
    }
    if (cg.status[q] != CG_PENDING) return;
    cg.checks[q] += 1;
    cg.true_res2[q] = tr;
    if (!isfinite(tr)) {
        cg.status[q] = CG_NAN;
    } else if (tr <= cg.tol2b[q]) {
        cg.status[q] = CG_CONVERGED;
    } else if (cg.iters[q] >= cg.max_iter) {
        cg.status[q] = CG_MAXITER;
    } else {
        cg.beta[q] = tr / cg.rho[q];
        cg.rho[q] = tr;
        cg.status[q] = CG_RESTART;
    }
}

// p = r + beta p for RHS restarting from a true residual.
__global__ __launch_bounds__(kBS) void k_cg_restart_p(int64_t n, const dvec2 *__restrict__ r,
                                                      dvec2 *__restrict__ p, CgDev cg) {
    const int rhs = blockIdx.y;
    if (cg.status[rhs] != CG_RESTART) return;
    const int64_t off = rhs * n;
    const double be = cg.beta[rhs];
    for (int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBS) {
        const dvec2 rr = r[off + i];
        dvec2 pp = p[off + i];
        pp.x = fma(be, pp.x, rr.x);
        pp.y = fma(be, pp.y, rr.y);
        p[off + i] = pp;
    }
}

// Restarted RHS become active again (after k_cg_restart_p has read their state).
__global__ __launch_bounds__(kBS) void k_cg_activate(int nrhs, CgDev cg) {
    const int q = blockIdx.x * kBS + threadIdx.x;
    if (q < nrhs && cg.status[q] == CG_RESTART) cg.status[q] = CG_ACTIVE;
}

}  // namespace

int blas_reduce_blocks(int64_t n) { return make_grid(n).nbx; }

#define AS_V(p) reinterpret_cast<dvec2 *>(p)
#define AS_CV(p) reinterpret_cast<const dvec2 *>(p)

hisq_status cg_init(int64_t n, int nrhs, const double2 *b, const double2 *Ax, double2 *r,
                    double2 *p, double tol, const CgDev &cg, const Reduce &red,
                    hipStream_t s) {
    const BlasGrid gr = make_grid(n);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_cg_init, dim3(gr.nbx, nrhs), dim3(kBS), 0, s, n, nrhs, AS_CV(b),
                       AS_CV(Ax), AS_V(r), AS_V(p), red.partials);
    HISQ_HIP(hipGetLastError());
    const int per = kBS / kWave;
    hipLaunchKernelGGL(k_cg_init_state, dim3((nrhs + per - 1) / per), dim3(kBS), 0, s, nrhs,
                       red.partials, gr.nbx, tol, cg);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status cg_update_r(int64_t n, int nrhs, double2 *r, const double2 *Ap, const double *pap,
                        int nb_pap, const CgDev &cg, const Reduce &red, hipStream_t s) {
    const BlasGrid gr = make_grid(n);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_cg_update_r<dvec2>, dim3(gr.nbx, nrhs), dim3(kBS), 0, s, n, AS_V(r),
                       AS_CV(Ap), pap, nb_pap, cg, red);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status cg_sum_pap(int nrhs, const double *pap, int nb_pap, double *pq, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_pap, dim3(nrhs), dim3(kSumBS), 0, s, pap, nb_pap, pq);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status cg_finalize(int64_t n, int nrhs, const double *pap, int nb_pap, const CgDev &cg,
                        const Reduce &red, hipStream_t s) {
    const BlasGrid gr = make_grid(n);
    ProfileScope prof("blas", s);
    const int per = kBS / kWave;
    hipLaunchKernelGGL(k_cg_finalize, dim3((nrhs + per - 1) / per), dim3(kBS), 0, s, nrhs, pap,
                       nb_pap, gr.nbx, cg, red);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status cg_update_xp(int64_t n, int nrhs, double2 *x, const double2 *r, double2 *p,
                         const CgDev &cg, hipStream_t s) {
    const BlasGrid gr = make_grid(n);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_cg_update_xp<dvec2>, dim3(gr.nbx, nrhs), dim3(kBS), 0, s, n, AS_V(x),
                       AS_CV(r), AS_V(p), cg);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

#define AS_F(p) reinterpret_cast<fvec2 *>(p)
#define AS_CF(p) reinterpret_cast<const fvec2 *>(p)

hisq_status cg_update_r(int64_t n, int nrhs, float2 *r, const float2 *Ap, const double *pap,
                        int nb_pap, const CgDev &cg, const Reduce &red, hipStream_t s) {
    const BlasGrid gr = make_grid(n);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_cg_update_r<fvec2>, dim3(gr.nbx, nrhs), dim3(kBS), 0, s, n, AS_F(r),
                       AS_CF(Ap), pap, nb_pap, cg, red);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status cg_update_xp(int64_t n, int nrhs, float2 *x, const float2 *r, float2 *p,
                         const CgDev &cg, hipStream_t s) {
    const BlasGrid gr = make_grid(n);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_cg_update_xp<fvec2>, dim3(gr.nbx, nrhs), dim3(kBS), 0, s, n, AS_F(x),
                       AS_CF(r), AS_F(p), cg);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status cg_true_residual(int64_t n, int nrhs, const double2 *b, const double2 *Ax,
                             double2 *r, const CgDev &cg, const Reduce &red, bool final_only,
                             hipStream_t s) {
    const BlasGrid gr = make_grid(n);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_cg_true_residual, dim3(gr.nbx, nrhs), dim3(kBS), 0, s, n, AS_CV(b),
                       AS_CV(Ax), AS_V(r), cg, red.partials, final_only ? 1 : 0);
    HISQ_HIP(hipGetLastError());
    const int per = kBS / kWave;
    hipLaunchKernelGGL(k_cg_true_state, dim3((nrhs + per - 1) / per), dim3(kBS), 0, s, nrhs,
                       red.partials, gr.nbx, cg, final_only ? 1 : 0);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status cg_restart_p(int64_t n, int nrhs, const double2 *r, double2 *p, const CgDev &cg,
                         hipStream_t s) {
    const BlasGrid gr = make_grid(n);
    ProfileScope prof("blas", s);
    hipLaunchKernelGGL(k_cg_restart_p, dim3(gr.nbx, nrhs), dim3(kBS), 0, s, n, AS_CV(r), AS_V(p),
                       cg);
    HISQ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cg_activate, dim3((nrhs + kBS - 1) / kBS), dim3(kBS), 0, s, nrhs, cg);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

}  // namespace hisq
