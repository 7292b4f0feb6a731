/*
 * hisq.h - C ABI of libhisq: the even-odd preconditioned HISQ solve on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operation is the one stated in arXiv:2502.00152, section 2: propagators
 * psi solve M psi = eta with M = D + 2m, D the anti-Hermitian HISQ matrix; the
 * normal equation M^H M psi = M^H eta (Eq. (1)) is solved by even-odd (Schur)
 * preconditioned conjugate gradient on the even sites,
 *
 *     A psi_e = y_e,   A = (2m)^2 - D_eo D_oe,   y_e = 2m eta_e - D_eo eta_o,
 *
 * the odd half follows as psi_o = (eta_o - D_oe psi_e) / (2m), and the CG can
 * start from the low-mode deflation guess x0 = sum_i v_i v_i^H b / lambda_i
 * (Eq. (4)) built from eigenpairs of A computed by thick-restart Lanczos
 * (section 2, the eigensolver paragraph).  The stencil is
 *
 *   (D psi)(x) = sum_mu [ F_mu(x) psi(x+mu) - F_mu(x-mu)^H psi(x-mu)
 *                       + L_mu(x) psi(x+3mu) - L_mu(x-3mu)^H psi(x-3mu) ]
 *
 * with F the fat links and L the long (Naik) links, coordinates periodic,
 * and no factor 1/2.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - dims = {X, Y, Z, T}; every extent even and >= 2.  Lexicographic site
 *    index lex = ((t*Z + z)*Y + y)*X + x; parity = (x+y+z+t) mod 2;
 *    checkerboard index cb = lex >> 1, 0 <= cb < Vh = X*Y*Z*T/2.
 *  - A "parity vector" (even or odd) is complex double, SoA layout
 *    [nrhs][3 colours][Vh], each complex stored as (re, im) doubles: element
 *    (r, c, cb) sits at byte offset 16*((r*3 + c)*Vh + cb).
 *  - A "full vector" is complex double [nrhs][T][Z][Y][X][3] (canonical).
 *  - Every pointer argument named *_dev is device memory (hipMalloc'd or a
 *    torch CUDA tensor), 16-byte aligned, owned by the caller, and not retained
 *    after the call returns.  Host arrays are named *_host.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it.  Calls that return host values
 *    (cg_solve, eigensolve, stats) synchronise that stream before returning.
 *  - Calls on one gauge handle must not overlap (the handle owns scratch
 *    buffers); different handles are independent.
 *  - Every call returns a hisq_status and never throws.  On a non-OK status,
 *    hisq_last_error() returns a message for the calling thread.
 */
#ifndef HISQ_H
#define HISQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hisq_status {
    HISQ_OK = 0,
    HISQ_ERR_INVALID_ARG = 1,  /* bad extent, size, pointer, parity or parameter */
    HISQ_ERR_HIP = 2,          /* a HIP runtime call failed */
    HISQ_ERR_OOM = 3,          /* device allocation failed */
    HISQ_ERR_NOT_CONVERGED = 4,/* iteration limit reached; best iterate returned */
    HISQ_ERR_NAN = 5,          /* NaN or Inf met in a residual or a reduction */
    HISQ_ERR_BREAKDOWN = 6,    /* <p, A p> <= 0 in CG, or an invariant Krylov space
                                  smaller than requested in the eigensolver */
    HISQ_ERR_UNSUPPORTED = 7   /* valid request that this build does not implement */
} hisq_status;

/* HISQ_Q16: 16-bit fixed-point links (one scale per gauge handle: the largest
 * link component / 32767) with FP32 vectors and arithmetic, for the stencil,
 * M^H M and the CG's sloppy operator only.
 * HISQ_HALF: the CG's search direction p, A p and the odd temporary held in
 * 16-bit fixed point with one scale per RHS and site (the largest |component|
 * of its three colours; relative accuracy ~3e-5), and links in 16-bit fixed
 * point with components up to qmax (scale: the largest link component / qmax),
 * qmax = min(32767, floor(65535 * largest component / largest row sum of
 * |Re| + |Im|) - 1), at least 10922 (~26700 for near-unitary links), so that
 * the stencil sums the integer products of a link row and a colour vector
 * exactly in 32 bits for any vector; for sloppy_prec and,
 * with FP32 vectors at the boundary, for hisq_dslash_eo and hisq_mdagm. */
typedef enum hisq_prec {
    HISQ_FP64 = 0,
    HISQ_FP32 = 1,
    HISQ_BF16 = 2,
    HISQ_Q16 = 3,
    HISQ_HALF = 4
} hisq_prec;

/* hisq_gauge_create flags */
enum {
    HISQ_GAUGE_FOLD_PHASES = 1u,     /* multiply link mu at x by the staggered phase
                                        eta_mu(x): 1, (-1)^x, (-1)^(x+y), (-1)^(x+y+z) */
    HISQ_GAUGE_ANTIPERIODIC_T = 2u   /* multiply a time link of hop h at t by
                                        (-1)^floor((t+h)/T) (antiperiodic fermions) */
};

typedef struct hisq_gauge_s *hisq_gauge;

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *hisq_last_error(void);

/* ABI revision of this header; bumped on any incompatible change. */
int hisq_abi_version(void);
#define HISQ_ABI_VERSION 10

/* ------------------------------------------------------------------ gauge */

/*
 * Build a gauge handle from fat links F and long links L (section 2: the HISQ
 * matrix; the stencil is written out at the top of this file).
 *   dims        {X, Y, Z, T}, even, >= 2, with X*Y*Z*T/2 < 2^31.
 *   fat_dev,    complex double [4][T][Z][Y][X][3][3] (row-major colour matrix,
 *   long_dev    mu = x, y, z, t); device memory, read only during the call.
 *   c_fat,      scalar factors applied to the fat and long links.
 *   c_long
 *   flags       HISQ_GAUGE_* bits: fold staggered phases and the antiperiodic
 *               time sign into the stored links.  Pass 0 (and 1.0, 1.0) for
 *               links that already carry everything.
 * The links are copied into the handle in the layout the kernels use; the
 * caller's buffers may be freed afterwards.  Errors: INVALID_ARG for bad
 * dims/pointers, OOM, HIP.
 */
hisq_status hisq_gauge_create(hisq_gauge *out, const int dims[4], const void *fat_dev,
                              const void *long_dev, double c_fat, double c_long,
                              unsigned flags, void *stream);

/* Release the handle and every buffer it owns (synchronises the device). */
hisq_status hisq_gauge_destroy(hisq_gauge g);

/* Vh = X*Y*Z*T/2 of the handle (0 for a NULL handle). */
int64_t hisq_gauge_half_volume(hisq_gauge g);

/* ---------------------------------------------------------------- layouts */

/*
 * Split full vectors [nrhs][T][Z][Y][X][3] into even and odd parity vectors
 * (layout above).  Either output may be NULL to skip it.
 */
hisq_status hisq_spinor_split(hisq_gauge g, const void *full_dev, void *even_dev,
                              void *odd_dev, int nrhs, void *stream);

/* Inverse of hisq_spinor_split.  A NULL input parity writes zeros there. */
hisq_status hisq_spinor_merge(hisq_gauge g, const void *even_dev, const void *odd_dev,
                              void *full_dev, int nrhs, void *stream);

/*
 * Change the precision of n_complex complex numbers (any vectors, e.g. the
 * eigenvectors stored in single precision for multi-deflation, section 3):
 * a narrowing conversion (HISQ_FP64 -> HISQ_FP32 or HISQ_BF16, HISQ_FP32 ->
 * HISQ_BF16) rounds to nearest even (FP64 -> BF16 in one rounding), a
 * widening one is exact, equal precisions copy.  HISQ_BF16 vectors hold a
 * complex number as two bfloat16 (real part first, 4 bytes).  src and dst
 * must not overlap.  Asynchronous
 * on `stream`.  INVALID_ARG for NULL or overlapping buffers, n_complex < 0 or
 * an unsupported precision.
 */
hisq_status hisq_convert_vectors(const void *src_dev, hisq_prec src_prec, void *dst_dev,
                                 hisq_prec dst_prec, int64_t n_complex, void *stream);

/* ------------------------------------------------------------- operators */

/*
 * Half stencil: out = D_{p,1-p} in for output parity p = out_parity
 * (0 = even: D_eo, odd -> even; 1 = odd: D_oe, even -> odd).  `in` is a parity
 * vector of parity 1-p, `out` of parity p; they must not overlap.
 * Section 2 (the HISQ matrix D; even-odd split).  prec: HISQ_FP64 (vectors
 * of complex double) or HISQ_FP32 (vectors of complex float, same layout,
 * 8 bytes per complex; FP32 links and FP32 arithmetic, the FP32 links made
 * from the FP64 ones on first use) or HISQ_BF16 (vectors of bfloat16 pairs,
 * 4 bytes per complex; BF16 links, FP32 arithmetic, each output rounded to
 * nearest even once; the BF16 links made from the FP64 ones on first use) or
 * HISQ_Q16 (vectors of complex float as for HISQ_FP32; links in 16-bit fixed
 * point, made from the FP64 ones on first use: absolute error <= step / 2 per
 * component, step = the largest link component of the handle / 32767) or
 * HISQ_HALF (vectors of complex float at the boundary; inside, the input is
 * rounded to 16-bit fixed point with one norm per RHS and site, the stencil of
 * the CG at sloppy_prec = HISQ_HALF is applied, with its links, and its
 * 16-bit output is widened to FP32: each value is that of the stored 16-bit
 * result).
 */
hisq_status hisq_dslash_eo(hisq_gauge g, int out_parity, const void *in_dev,
                           void *out_dev, int nrhs, hisq_prec prec, void *stream);

/*
 * Even-site normal operator: out_e = ((2m)^2 - D_eo D_oe) in_e, the even-even
 * block of M^H M (Eq. (1) after even-odd preconditioning).  two_m = 2m >= 0.
 * in_e and out_e must not overlap.  Uses an odd-parity scratch vector owned by
 * the handle.  prec as for hisq_dslash_eo.
 */
hisq_status hisq_mdagm(hisq_gauge g, double two_m, const void *in_e_dev, void *out_e_dev,
                       int nrhs, hisq_prec prec, void *stream);

/* Bytes of the device array that hisq_mdagm_noalloc uses as its scratch. */
#define HISQ_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * hisq_mdagm for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that
 * forbid allocation.  Same operator, kernels and launch shapes as hisq_mdagm
 * (the same results bit for bit), but its odd-parity temporary lives in one
 * file-scope device array of HISQ_NOALLOC_SCRATCH_BYTES per GPU (held until
 * the process ends) instead of the handle's scratch, and the call makes no
 * allocation of any kind (no hipMalloc, hipFree, event or library buffer;
 * kernel timing by hisq_profile_enable is skipped for it).  The caller owns
 * in_e and out_e as for hisq_mdagm; the device current on the calling thread
 * must be the handle's.
 * prec: HISQ_FP64, or HISQ_FP32 once the handle's FP32 links exist (a first
 * hisq_mdagm or hisq_dslash_eo call with HISQ_FP32 makes them; otherwise
 * HISQ_ERR_INVALID_ARG).  The temporary takes 3 * Vh * nrhs complex numbers
 * of prec (48 or 24 bytes per site and RHS); a call that needs more than
 * HISQ_NOALLOC_SCRATCH_BYTES returns HISQ_ERR_INVALID_ARG and launches
 * nothing.  Every call on one GPU shares that GPU's array: calls that overlap
 * in time on one GPU (two streams, two threads) race and give wrong results;
 * the array keeps the last call's contents, which no later call reads before
 * writing it.
 */
hisq_status hisq_mdagm_noalloc(hisq_gauge g, double two_m, const void *in_e_dev,
                               void *out_e_dev, int nrhs, hisq_prec prec, void *stream);

/*
 * Even-site source of the preconditioned system: y_e = 2m eta_e - D_eo eta_o,
 * the even half of M^H eta (section 2, the Schur step before the CG).
 */
hisq_status hisq_prepare_source(hisq_gauge g, double two_m, const void *eta_e_dev,
                                const void *eta_o_dev, void *y_e_dev, int nrhs,
                                void *stream);

/*
 * Odd half of the solution from the odd rows of M psi = eta:
 * psi_o = (eta_o - D_oe psi_e) / (2m).  two_m > 0.  (Section 2 prints this
 * step garbled; this is the form under which M psi = eta holds exactly.)
 */
hisq_status hisq_reconstruct_odd(hisq_gauge g, double two_m, const void *psi_e_dev,
                                 const void *eta_o_dev, void *psi_o_dev, int nrhs,
                                 void *stream);

/* ------------------------------------------------------------------- CG */

typedef struct hisq_cg_params {
    double tol;            /* stop when ||b - A x|| / ||b|| <= tol (true residual, FP64) */
    int max_iter;          /* iteration limit per right-hand side */
    int check_interval;    /* iterations between host polls of the convergence state
                              (0 = default 16).  It does not change the iterates of the
                              FP64 solve. */
    hisq_prec sloppy_prec; /* HISQ_FP64: plain FP64 CG.  HISQ_FP32: mixed precision,
                              the iteration in FP32 with FP64 reliable updates.
                              HISQ_BF16 / HISQ_Q16: the same with the sloppy
                              operator reading BF16 / 16-bit fixed-point links
                              (vectors still FP32).  HISQ_HALF: 16-bit links and
                              16-bit p, A p (residual and correction FP32) */
    int reliable_interval; /* mixed only: also a reliable update after this many
                              iterations since the last one (0 = only the delta
                              trigger, as in the paper) */
    double reliable_delta; /* mixed only: reliable update when the iterated residual
                              falls below reliable_delta times the true residual of
                              the last update (0 = default 0.1, the paper's delta_rd) */
    /* multi-deflation (section 3): re-deflate the residual during the solve */
    int n_ev;              /* 0: no re-deflation */
    hisq_prec evec_prec;   /* HISQ_FP64 or HISQ_FP32 eigenvectors */
    const void *evecs_dev; /* n_ev even parity vectors (layout of hisq_deflate) */
    const double *evals_host; /* eps_i of the massless operator, n_ev doubles */
    double tol_restart;    /* re-deflate at a reliable update when the true residual has
                              fallen by this factor since the last deflation
                              (the paper's delta_tr, e.g. 1e-3; 0 = never) */
    const double *two_m_rhs; /* optional host array of nrhs masses 2m, one per
                              right-hand side (several masses in one batched
                              solve, sharing every link load); replaces the
                              two_m argument; not with re-deflation */
    int parity;            /* 0: the even system A = (2m)^2 - D_eo D_oe (default);
                              1: the odd one, (2m)^2 - D_oe D_eo = (M^H M)_oo, used
                              to polish the reconstructed odd solution (section 2);
                              re-deflation needs parity 0 */
    int reserved[7];       /* must be zero */
} hisq_cg_params;

typedef struct hisq_cg_stats {
    int iterations;        /* operator applications inside the loop */
    int true_residual_checks; /* recomputations of b - A x (after the initial one) */
    int converged;         /* 1 if the true residual met tol */
    int reliable_updates;  /* FP64 true-residual replacements of the sloppy residual */
    int redeflations;      /* deflations of the residual during the solve */
    int reserved0;
    double true_residual;  /* final ||b - A x|| / ||b||, FP64 */
    double b_norm;         /* ||b|| */
} hisq_cg_stats;

/*
 * Solve A x = b on even sites, A = (2m)^2 - D_eo D_oe, for nrhs right-hand
 * sides at once (section 2: the even-odd preconditioned CG, the paper's
 * baseline; Eq. (1)); with params->parity = 1 the odd system
 * ((2m)^2 - D_oe D_eo) x_o = b_o instead (vectors of odd parity).  x_e_dev holds the initial guess on entry (zeros, or a
 * deflation guess from hisq_deflate) and the solution on return.  Each
 * right-hand side follows its own CG recurrence with FP64 global reductions
 * in a fixed order, so results are bitwise reproducible run to run.  A
 * right-hand side stops when its iterated residual crosses tol and the
 * recomputed true residual confirms it; if the true residual does not, CG
 * continues from it with the search direction kept.  b = 0 gives x = 0.
 *   stats_host: array of nrhs structs, filled on return (may be NULL).
 * With sloppy_prec = HISQ_FP32, HISQ_BF16, HISQ_Q16 or HISQ_HALF (section 2: the conventional solve is
 * mixed-precision CG; reliable updates as in section 3) the recurrence runs
 * on FP32 vectors with the FP32 operator and FP64-accumulated dot products;
 * the solution accumulates in FP64, and a reliable update (x += x_sloppy,
 * r = b - A x in FP64) follows whenever the iterated residual has fallen by
 * reliable_delta since the last one (and, if set, every reliable_interval
 * iterations), and before any convergence decision.  With n_ev > 0 and tol_restart > 0 the residual is
 * re-deflated, x += V diag(1/(eps + (2m)^2)) V^H r, when the true residual has
 * fallen by tol_restart since the last deflation, and the recurrence restarts
 * (section 3: multi-deflation with single-precision eigenvectors).
 * Returns NOT_CONVERGED if any right-hand side hit max_iter (x holds its last
 * iterate), NAN, BREAKDOWN, or INVALID_ARG (two_m <= 0, tol <= 0, ...).
 * Synchronises `stream`.
 */
hisq_status hisq_cg_solve(hisq_gauge g, double two_m, const void *b_e_dev, void *x_e_dev,
                          int nrhs, const hisq_cg_params *params,
                          hisq_cg_stats *stats_host, void *stream);

/* ------------------------------------------------------------ deflation */

/*
 * Deflation guess x0 = V diag(1 / (eps_i + (2m)^2)) V^H b (Eq. (4)), where the
 * columns of V are orthonormal even-site eigenvectors of the massless
 * operator -D_eo D_oe with eigenvalues eps_i (Eq. (3): the massive eigenvalue
 * is eps_i + (2m)^2 and the vectors do not depend on m).
 *   evecs_dev       n_ev even parity vectors [n_ev][3][Vh], complex double
 *                   (evec_prec = HISQ_FP64) or complex float (HISQ_FP32: the
 *                   single-precision eigenvectors of section 3).
 *   evals_host      eps_i, n_ev doubles (host); eps_i + (2m)^2 must be > 0.
 *   b_e_dev, x0_e_dev  complex double parity vectors with nrhs right-hand sides;
 *                   must not overlap.
 * The two contractions run on the FP64 matrix cores (FP32 eigenvectors are
 * widened on load; coefficients are FP64).
 */
hisq_status hisq_deflate(hisq_gauge g, int n_ev, const void *evecs_dev, hisq_prec evec_prec,
                         const double *evals_host, double two_m, const void *b_e_dev,
                         void *x0_e_dev, int nrhs, void *stream);

/* ------------------------------------------------- many systems at once */

typedef struct hisq_system {
    hisq_gauge g;          /* lattice and links of this system */
    double two_m;          /* its mass */
    const void *b_dev;     /* [nrhs][3][Vh] right-hand sides (parity of params) */
    void *x_dev;           /* [nrhs][3][Vh] initial guess in, solution out */
    int nrhs;
    int reserved;          /* must be zero */
} hisq_system;

/*
 * Solve n_systems independent systems (different lattices, masses and
 * numbers of RHS; the paper's future-work batching of uneven solves, section
 * 4) concurrently: systems on different gauge handles run at the same time,
 * each on its handle's own stream driven by its own host thread; systems
 * sharing a handle run one after another.  Each system follows exactly the
 * iterates of hisq_cg_solve with params[i] (bitwise), so only the wall time
 * changes.
 *   params      n_systems parameter sets (one per system).
 *   stats_host  sum of nrhs structs, the systems' in order (may be NULL).
 * Returns the first failing system's status (its message names it).
 * Synchronises.
 */
hisq_status hisq_cg_solve_multi(int n_systems, const hisq_system *systems,
                                const hisq_cg_params *params, hisq_cg_stats *stats_host,
                                void *stream);

/* ------------------------------------------------------ full propagator */

typedef struct hisq_prop_params {
    hisq_cg_params cg;     /* the even solve; with cg.n_ev > 0 the eigenvectors also
                              give the initial guess (Eq. (4)) */
    double polish_tol;     /* > 0: polish the reconstructed odd solution by CG on
                              (M^H M)_oo psi_o = (M^H eta)_o to this tolerance,
                              from psi_o (section 2's workflow); 0: no polish */
    int polish_max_iter;   /* 0 = cg.max_iter */
    int reserved[7];       /* must be zero */
} hisq_prop_params;

typedef struct hisq_prop_stats {
    hisq_cg_stats even;    /* the even CG */
    hisq_cg_stats polish;  /* the odd polish CG (zero if none) */
    double residual;       /* ||eta - M psi|| / ||eta|| over the full lattice, FP64 */
    double residual_even;  /* the even rows' part of it (the odd rows vanish before
                              the polish) */
    double reserved[2];
} hisq_prop_stats;

/*
 * Full propagator solve of M psi = eta, M = D + 2m, for nrhs full-lattice
 * sources (e.g. 3 colours x 2 propagators, the paper's workflow in section
 * 2): split eta, y_e = (M^H eta)_e, optional deflation guess, CG on the even
 * system (FP64 or mixed precision, with re-deflation, per params->cg),
 * psi_o = (eta_o - D_oe psi_e) / (2m), optional odd polish, merge, and the
 * final FP64 residual.
 *   eta_dev, psi_dev  [nrhs][T][Z][Y][X][3] complex double, device; must not
 *                     overlap.
 *   stats_host        nrhs structs (may be NULL).
 * Returns the status of the first failing stage (NOT_CONVERGED etc., with psi
 * holding the last iterate), INVALID_ARG for bad arguments.  Synchronises.
 */
hisq_status hisq_propagator_solve(hisq_gauge g, double two_m, const void *eta_dev, void *psi_dev,
                                  int nrhs, const hisq_prop_params *params,
                                  hisq_prop_stats *stats_host, void *stream);

/* --------------------------------------------------------- eigensolver */

/*
 * Progress report of hisq_eigensolve, called on the calling thread after each
 * Lanczos step: restart = -1 during the pilot, else the restart count; step =
 * the basis index just completed; matvecs = applications of A so far;
 * seconds = wall time since the call began.  It must not call the library.
 */
typedef void (*hisq_eig_progress_fn)(void *user, int restart, int step, int matvecs,
                                     double seconds);

typedef struct hisq_eig_params {
    int n_kr;              /* Krylov basis size (0 = auto: max(2*n_ev, n_ev + 32),
                              rounded up to a multiple of the block size) */
    int cheb_degree;       /* Chebyshev filter degree (0 = auto) */
    double cheb_a;         /* filter interval [a, b] of A to suppress (0 = auto) */
    double cheb_b;
    double tol;            /* accept when ||A v - lambda v|| <= tol * lambda_max(A) */
    int max_restarts;      /* 0 = default 200 */
    int evec_prec;         /* storage of evecs_dev: HISQ_FP64 (0) or HISQ_FP32 (the
                              solve itself is FP64 throughout; FP32 output is the
                              FP64 result rounded, section 3's single-precision
                              eigenvectors) */
    uint64_t seed;         /* seed of the counter-based start vector */
    hisq_eig_progress_fn progress; /* optional progress report (NULL: none) */
    void *progress_user;   /* passed to progress */
    int block;             /* Lanczos block size nb (0 or 1: one vector per step;
                              at most 32): each step filters nb vectors in one
                              multi-RHS stencil launch per half stencil (block
                              thick-restart Lanczos, the block variant named in
                              the conclusions); needs
                              n_ev + 2 nb - 1 <= n_kr <= 3 Vh - nb */
    int reserved[7];       /* must be zero */
} hisq_eig_params;

typedef struct hisq_eig_stats {
    int restarts;
    int matvecs;           /* applications of A (each = two half stencils) */
    int converged;         /* number of accepted pairs (n_ev on success) */
    int cheb_degree;
    double cheb_a, cheb_b;
    double lambda_max;     /* estimated largest eigenvalue of A */
    double max_residual;   /* max_i ||A v_i - lambda_i v_i|| after Rayleigh-Ritz */
    double seconds;
} hisq_eig_stats;

/*
 * Lowest n_ev eigenpairs of A = (2m)^2 - D_eo D_oe on even sites by
 * thick-restart Lanczos on a Chebyshev-filtered A, ending with a Rayleigh-Ritz
 * step on A itself (section 2: eigenvectors of the squared operator from
 * thick-restart Lanczos, used for deflation; the vectors are single parity,
 * section 3).
 *   evecs_dev   caller-allocated [n_ev][3][Vh] complex double, or complex float
 *               with evec_prec = HISQ_FP32 (orthonormal on exit)
 * Device memory: one FP64 basis of n_kr + nb vectors, a block of
 * max(min(n_ev, 32), nb) vectors (twice: the block and M^H M's odd
 * temporary) and four blocks of nb vectors (48 Vh bytes each), freed before
 * the call returns (M^H M's temporary stays with the gauge's scratch); e.g.
 * n_ev = 512, n_kr = 640, nb = 1 at 48^3 x 96 (Vh = 5308416) takes 173 GB
 * besides the caller's 65 GB of FP32 eigenvectors and the links.
 *   evals_host  n_ev doubles, ascending: eigenvalues of A at this two_m
 *   stats_host  may be NULL.
 * Returns NOT_CONVERGED if max_restarts passes without n_ev accepted pairs
 * (the best Ritz pairs are still written), BREAKDOWN, INVALID_ARG
 * (n_ev < 1, block outside [0, 32], n_kr outside the range above), OOM.
 * Synchronises `stream`.
 */
hisq_status hisq_eigensolve(hisq_gauge g, double two_m, int n_ev,
                            const hisq_eig_params *params, void *evecs_dev,
                            double *evals_host, hisq_eig_stats *stats_host, void *stream);

/* ------------------------------------------------------------- tuning */

/*
 * Launch-shape knobs of the kernels, process-wide (for the autotuner and for
 * measurements); results do not depend on them, only speed, except where a
 * key says otherwise.  Keys:
 *   "dslash_rhs_per_thread"  right-hand sides one lane carries: 0 = automatic,
 *                            or one of 1, 2, 3, 4, 6, 12
 *   "dslash_lanes_per_site"  lanes that share one site's link loads, each with
 *                            its own RHS: 0 = automatic, 1, 2 or 4 (with 2 or 4,
 *                            rhs_per_thread must be 1, 3 or 6; otherwise the
 *                            stencil calls return INVALID_ARG)
 *   "dslash_group_order"     -1: automatic; 0: RHS groups of one site block run
 *                            next to each other; 1: all sites of one group first
 *   "dslash_xcd_remap"       -1: automatic (3 or more RHS above 2^18 sites
 *                            per parity: chunks of an eighth of a time slice;
 *                            otherwise contiguous ranges, or dispatch order
 *                            for 1-2 RHS in FP32); 1: give each XCD a
 *                            contiguous range of sites; 0: dispatch order;
 *                            n >= 2: deal chunks of n launched blocks (site
 *                            blocks x RHS groups) round-robin to the XCDs
 *   "dslash_march"           -1: automatic (off); 0: off; n > 0: for two or
 *                            more RHS when X Y Z / 2 is a multiple of 256, the
 *                            kernel that marches along time with n time
 *                            segments: each workgroup takes 256 sites of a
 *                            slice and keeps their time neighbours in
 *                            registers (FP64, FP32 and 16-bit storage; never
 *                            BF16); bitwise the same results
 *   "dslash_blocks_per_cu"   -1: automatic (3 for FP32 vectors with 12 or more
 *                            RHS above 2^18 sites per parity, else no cap;
 *                            or the autotuner's choice); 0: no cap; 1-8: each
 *                            stencil launch requests enough (unused) LDS that
 *                            at most this many of its blocks share a compute
 *                            unit, fewer sites in flight per XCD (measured at
 *                            48^3 x 96, 12 RHS: FP32 vectors 3.57 -> 3.34 ms
 *                            with 3; the 16-bit CG stencil gains nothing)
 *   "dslash_autotune_clear"  any value: forget the autotuner's choices
 *   "gemm_fp32_mfma"         -1: automatic; 0: never; 1: always: the projection
 *                            with FP32 eigenvectors (V^H B and V C) on the FP32
 *                            matrix cores (products in FP32, each wave's part of
 *                            a sum in FP32, the parts summed in FP64) instead of
 *                            widening to FP64; automatic: where the FP64 form
 *                            would be bound by the FP64 matrix rate (4 k n /
 *                            (4 k + 8 n) > 10 flop/B, e.g. 256 vectors x 24 RHS).
 *                            This knob changes results at the FP32 rounding level.
 *   "cg_reliable_freeze"     mixed CG: -1 automatic (on for sloppy_prec
 *                            HISQ_BF16 only); 1: a right-hand side
 *                            whose iterated residual has fallen by
 *                            reliable_delta stops iterating until its
 *                            reliable update at the next host poll; 0: it
 *                            iterates on until then.  Changes iterates and
 *                            iteration counts.
 *   "cg_multi_graph"         -1 automatic (off), 0 off, 1: hisq_cg_solve_multi
 *                            launches each chunk of iterations of all systems
 *                            (on distinct gauge handles) as one captured HIP
 *                            graph, the systems' kernels on parallel branches
 *                            (bitwise the same results as separate streams)
 *   "cg_graphs"              -1 automatic (off), 0 off, 1: replay the CG's
 *                            chunks of iterations from a captured HIP graph
 *                            (measured: no gain on MI355X, kept as an option)
 * The <aux, out> partial sums of the CG are formed in one fixed order for any
 * shape, so CG iterates are bitwise independent of these knobs too.
 * Returns INVALID_ARG for an unknown key or value.
 */
hisq_status hisq_set_tuning(const char *key, int64_t value);

typedef struct hisq_tune_result {
    int rhs_per_thread;    /* the chosen shape */
    int lanes_per_site;
    int group_order;
    int xcd_remap;
    double us_best;        /* average launch time of the chosen shape */
    double us_default;     /* and of the shape in use before the call */
    int shapes_timed;
    int march;             /* time segments of the time-marching kernel (0: not used) */
    int blocks_per_cu;     /* cap on blocks per compute unit (0: none) */
    int reserved[1];
} hisq_tune_result;

/*
 * Autotuner of the half stencil: time every launch shape the kernel provides
 * (RHS per lane x lanes per site x block order x XCD remap, then a cap of 4,
 * 3 or 2 blocks per compute unit on the fastest) for this handle's
 * volume, nrhs right-hand sides and precision prec (HISQ_FP64 or HISQ_FP32),
 * `reps` launches each (0 = 20) on scratch vectors, with HIP events on
 * `stream`; remember the fastest for (volume, nrhs, prec) for the rest of the
 * process (every later stencil, M^H M, CG and eigensolver launch of that size
 * uses it, unless a "dslash_*" knob is set).  Results do not change, only
 * speed.  Leaves the "dslash_*" knobs at automatic.  Not safe to run
 * concurrently with other library calls.
 * Synchronises; result_host may be NULL.
 */
hisq_status hisq_autotune_dslash(hisq_gauge g, int nrhs, hisq_prec prec, int reps,
                                 hisq_tune_result *result_host, void *stream);

/* ------------------------------------------------- learned initial guess */

/*
 * A small gauge-covariant network N that maps the residual r0 = b - A x0 of an
 * initial guess x0 (normally the deflation guess of Eq. (4)) to a correction
 * of it.  This goes beyond arXiv:2502.00152, whose solver is deflated CG
 * (section 2): CG stays the solver with its true-residual stop unchanged, and
 * hisq_nn_guess keeps a correction only for the RHS whose ||b - A x|| it lowers.
 *
 * N has HISQ_NN_CHANNELS = 8 channels, each a colour-vector field on every
 * site, and three layers
 *
 *   layer(W, psi)^o = sum_{d=0..8} sum_c W[d][o][c] T_d psi^c,
 *   T_0 = 1,  (T_{1+mu} psi)(x) = F_mu(x) psi(x+mu),
 *   (T_{5+mu} psi)(x) = F_mu(x-mu)^H psi(x-mu)
 *
 * (F: the handle's fat links with their folded phases, rounded to FP32; real
 * weights, so N commutes with gauge transformations) with norm gates
 *
 *   gate(g, psi)^c(x) = psi^c(x) / (1 + exp(-(a_c |psi^c(x)| + b_c)))
 *
 * between them: N(r) = even part of layer(W3, gate(g2, layer(W2, gate(g1,
 * layer(W1, r))))), with r on the even sites and zero on the odd ones.  The
 * HISQ_NN_PARAMS = 752 parameters are floats in the order W1 [9][8][1],
 * W2 [9][8][8], W3 [9][1][8], g1 [8][2] = (a_c, b_c), g2 [8][2], row-major.
 * Activations are FP32; gradients of weights and gates, norms and the loss are
 * summed in FP64 in a fixed order, so results repeat bit for bit.
 *
 * Flags: HISQ_NN_NORMALIZE - the network sees r_s / ||r_s|| and its output is
 * scaled back by ||r_s|| (per sample; the loss then compares with
 * e_s / ||r_s||).  HISQ_NN_BF16 - inference with the parameters rounded to
 * bfloat16 (nearest even), FP32 arithmetic (hisq_nn_apply, hisq_nn_guess).
 *
 * Even parity vectors use the layout of every other entry point; a batch of
 * nsamp of them is [nsamp][3][Vh] complex double.  A network handle belongs to
 * the gauge handle it was created on (which must outlive it); calls on one
 * network must not overlap.  The network owns its parameters, Adam moments
 * and activation scratch: 2448 * Vh bytes per sample in training (51 FP32
 * channel fields), 816 * Vh in inference.
 */
#define HISQ_NN_CHANNELS 8
#define HISQ_NN_PARAMS 752
enum { HISQ_NN_NORMALIZE = 1u, HISQ_NN_BF16 = 2u };

typedef struct hisq_nn_s *hisq_nn;

/* Create a network on g.  params_host: HISQ_NN_PARAMS finite floats, or NULL
 * for all zeros (N = 0).  Adam moments start at zero. */
hisq_status hisq_nn_create(hisq_nn *out, hisq_gauge g, const float *params_host);
hisq_status hisq_nn_destroy(hisq_nn n);  /* NULL is a no-op; synchronises */
/* Replace the parameters (and reset Adam); read them back.  Both synchronise. */
hisq_status hisq_nn_set_params(hisq_nn n, const float *params_host);
hisq_status hisq_nn_get_params(hisq_nn n, float *params_host);

/* out_s = N(r_s) for nsamp (1..4096) even vectors; out must not overlap r.
 * Enqueued on stream, no synchronisation. */
hisq_status hisq_nn_apply(hisq_nn n, const void *r_dev, void *out_dev, int nsamp,
                          unsigned flags, void *stream);

/* Loss of a batch, loss = (1/nsamp) sum_s ||N(r_s) - e_s||^2 / ||e_s||^2, and
 * its gradient with respect to the parameters (grad_host: HISQ_NN_PARAMS
 * doubles, or NULL; it is also kept for hisq_nn_adam_step).  e_s must be
 * nonzero (else HISQ_ERR_NAN).  FP32 parameters only (no HISQ_NN_BF16).
 * Synchronises. */
hisq_status hisq_nn_loss_grad(hisq_nn n, const void *r_dev, const void *e_dev, int nsamp,
                              unsigned flags, double *loss_host, double *grad_host,
                              void *stream);

/* One Adam step (Kingma and Ba) from the last gradient: t += 1,
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), in FP32.
 * INVALID_ARG before the first hisq_nn_loss_grad or for lr <= 0,
 * b outside [0, 1), eps <= 0. */
hisq_status hisq_nn_adam_step(hisq_nn n, double lr, double beta1, double beta2, double eps,
                              void *stream);

/* Train on npairs (r, e) pairs: `steps` Adam steps (beta1 0.9, beta2 0.999,
 * eps 1e-8); step k uses the mini-batch of `batch` consecutive pairs number
 * k mod floor(npairs / batch) (pairs past the last whole batch are unused).
 * loss_host[k] (steps doubles, or NULL) = the loss of step k's batch before
 * its update.  Synchronises. */
hisq_status hisq_nn_train(hisq_nn n, const void *r_dev, const void *e_dev, int npairs,
                          int batch, int steps, double lr, unsigned flags,
                          double *loss_host, void *stream);

/* The initial guess: for each RHS j, r = b_j - A x_j (A = (2m)^2 - D_eo D_oe,
 * FP64) and d = N(r); with n_ev > 0 eigenpairs (the arguments of
 * hisq_deflate: evecs_dev, evec_prec, evals_host = eps_i) the Galerkin
 * correction d += V diag(1/(eps_i + (2m)^2)) V^H (r - A d) follows, which
 * for a deflated x (V^H r = 0) removes the component of d in the deflation
 * space (without it, error put back into the lowest modes makes CG slower
 * than from the deflation guess alone).  Then x_j += d where
 * ||r - A d|| < ||r||.  n_ev = 0 skips the projection (evecs_dev and
 * evals_host are then not read).  kept_host (nrhs ints, or NULL) receives 1
 * where the correction was kept (then the call synchronises).  b and x must
 * not overlap. */
hisq_status hisq_nn_guess(hisq_nn n, double two_m, const void *b_dev, void *x_dev, int nrhs,
                          unsigned flags, int n_ev, const void *evecs_dev, hisq_prec evec_prec,
                          const double *evals_host, int *kept_host, void *stream);

/* ------------------------------------------------------ instrumentation */

/*
 * Per-kernel timing with HIP events recorded on the launch stream around
 * every launch of the named kernel class: "dslash" (plain half stencil),
 * "dslash_aux" (with one epilogue field: M^H M second half, source, odd
 * reconstruction), "dslash_aux2" (two epilogue fields: Chebyshev step),
 * "dslash_f32", "dslash_f32_aux", "dslash_f32_aux2" (the same in FP32), "blas"
 * (CG and Lanczos vector kernels), "gemm" (matrix-core contractions),
 * "nn_layer" (the learned guess's layer kernel, forward and backward); off by
 * default.  hisq_profile_enable(n): n = 0 off; n >= 1 times every n-th launch
 * of each class (counting from the call), so that a long run can be sampled
 * with few events in the stream; n < 0 is INVALID_ARG.  hisq_profile_read
 * returns the number of timed launches and their total milliseconds
 * (synchronises the device), and clears the record.
 */
hisq_status hisq_profile_enable(int on);
hisq_status hisq_profile_read(const char *kernel_class, int64_t *launches,
                              double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* HISQ_H */
