"""Benchmark of the HISQ deflated even-odd CG path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--budget-s S]
                    [--no-cpu-baseline] [--no-secondary] [--no-uneven]
                    [--no-dslash-scan] [--no-ru-variants] [--pmc-probe 48|16|32]
                    [--gemm-probe] [--eig-recipe]

Headline workload (the learned-guess configuration, synthetic): one GPU's
share of a large lattice, 48^3 x 96, random SU(3) fat and long links (eps 0.5,
long links scaled by -1/24, staggered phases and antiperiodic time folded
in), 2m = 0.002, 12 Gaussian sources per step, true-residual target 1e-10
(FP64 residual b - A x).

One step solves the 12 sources end to end on the GPU, inputs resident in HBM,
with the paper's production method (sections 2 and 3) plus the learned
guess: source preparation y_e = 2m eta_e - D_eo eta_o (FP64); deflation guess
x0 = V diag(1/lambda) V^H y_e with single-precision eigenvectors; the learned
correction (gauge-covariant network, BF16 weights, projected off the
deflation space, kept per source only where it lowers the FP64 residual);
batched mixed-precision CG (16-bit fixed-point links, search direction and
A p with a norm per site, FP32 residual and correction, FP64 dot products,
FP64 reliable updates at delta_rd = 0.1) with re-deflation whenever the true
residual has fallen by delta_tr = 1e-3 since the last deflation, to
||y - A x|| <= 1e-10 ||y||; odd reconstruction (FP64).  Setup (gauge packing),
the eigensolve (FP64) and the network's training (on pairs the solver
generates) are outside the timed region, as the paper times solves only;
all are timed and reported.  The eigensolve is block thick-restart Lanczos
(--eig-block vectors per step through the multi-RHS stencil).  value =
solves per second = 12 K / (K steps).

Also reported: the same step without the learned guess; the same sources in
FP64 throughout (FP64 eigenvectors, single deflation, FP64 CG) and each mixed
solution's difference from it; the oracle-evaluated FP64 residual of two
sources; the solve with the reliable update taken at three points (stopped
at the delta_rd trigger until the next host poll, run on to the poll, a poll
after every iteration); plain FP64 even-odd CG (no deflation, one source);
the live roofline
of the CG's 16-bit half stencil (HIP events inside the timed region); the
oracle timed on the host cores; and secondary legs: the 16^3 x 32 deflated
workload, the uneven batch (four lattices x three masses) and a half-stencil
scan at 32^3 x 64 and 48^3 x 96.  Legs after the headline are skipped once
the run has used --budget-s seconds.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s at 1e-10 true residual (learned+mixed+batched vs plain CG); Dslash GB/s"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed instructions (disabled in every kernel here):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# two-way int16 dot products (two multiply-adds per lane and cycle), the form
# the 16-bit stencil computes its products in: 157.3 T ops/s
DOT2_VALU_PEAK_TOPS = 2 * FP32_VALU_PEAK_TFLOPS
FP64_MFMA_PEAK_TFLOPS = 78.6
STENCIL_FLOPS_PER_SITE_RHS = 16 * 66 + 15 * 6  # 16 SU(3) x vector products and their sum
PROFILE_PERIOD = 16
T0 = time.perf_counter()


def say(msg):
    print(f"[bench {time.perf_counter() - T0:6.1f}s] {msg}", flush=True)


def dslash_alg_bytes(vh, nrhs, aux_fields, real_bytes=8, link_bytes=None, site_bytes=None):
    """Algorithmic HBM bytes of one half-stencil launch: 16 links of 18 reals
    per output site once, the input field once, the output once and each
    epilogue field once, per RHS (one colour vector = 6 reals per site).
    link_bytes: bytes per stored link real (default real_bytes); site_bytes:
    bytes of one RHS's colour vector at one site (default 6 real_bytes; 16 for
    16-bit vectors with their norm)."""
    lb = real_bytes if link_bytes is None else link_bytes
    sb = 6 * real_bytes if site_bytes is None else site_bytes
    return vh * (16 * 18 * lb + nrhs * sb * (2 + aux_fields))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("dslash_kernel.h", "dslash.hip", "dslash_f32.hip", "dslash_q16.hip", "cg_half.hip",
              "device_util.h"):
        with open(os.path.join(ROOT, "paper_2502_00152_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(name):
    """HBM traffic per half-stencil launch from a committed counter summary,
    if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def device_gauge(cfg):
    """Links drawn on the device (seeded), packed into a gauge handle; returns
    (handle, raw fat links, raw long links, pack seconds).  The raw links are
    kept on the host side only when the caller needs them for the oracle."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    W = I.random_su3_field_device(cfg["dims"], cfg["eps"], cfg["seed_fat"])
    N = I.random_su3_field_device(cfg["dims"], cfg["eps"], cfg["seed_long"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = hisq.Gauge(cfg["dims"], W, N, cfg["c_fat"], cfg["c_long"])
    torch.cuda.synchronize()
    return g, W, N, time.perf_counter() - t0


def device_sources(g, n, seed, two_m):
    """n Gaussian full-lattice sources drawn on the device, split into parities;
    returns (eta_e, eta_o)."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    ee = torch.randn((n, 3, g.vh), dtype=torch.complex128, device="cuda", generator=gen)
    eo = torch.randn((n, 3, g.vh), dtype=torch.complex128, device="cuda", generator=gen)
    return ee, eo


def eigensolve(g, two_m, n_ev, tol, seed, tag, block=0):
    import torch
    from paper_2502_00152_amd import hisq
    evecs = torch.empty((n_ev, 3, g.vh), dtype=torch.complex128, device="cuda")
    last = [0.0]

    def prog(r, j, mv, sec):
        if sec - last[0] >= 20.0:
            last[0] = sec
            say(f"{tag} eigensolve restart {r} step {j} matvecs {mv} {sec:.0f} s")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, lam, est = hisq.hisq_eigensolve(g, two_m, n_ev, evecs, tol=tol, seed=seed, progress=prog,
                                       block=block)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    say(f"{tag} eigensolve {t_eig:.1f} s, {est.matvecs} matvecs, {est.restarts} restarts, "
        f"block {max(block, 1)}, max residual {est.max_residual:.2e}, lambda_1 {lam[0]:.4e}")
    info = {"seconds": t_eig, "n_ev": n_ev, "tol": tol, "block": max(block, 1),
            "matvecs": est.matvecs,
            "restarts": est.restarts, "cheb_degree": est.cheb_degree,
            "max_residual": est.max_residual, "lambda_max": est.lambda_max,
            "lambda_1": float(lam[0]), f"lambda_{n_ev}": float(lam[-1])}
    return evecs, lam, info


def train_streamed(g, ev32, eps, two_m, n_pairs, nrhs, seed, steps_per_batch, lr=1e-2, batch=2):
    """The learned guess trained on pairs the production solver generates,
    streamed: each batch of nrhs pairs (r = residual of the deflation guess of
    a prepared random source, e = the remaining error from a 1e-12 solve) is
    trained on and dropped, so any number of pairs fits in memory."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    net = hisq.Network(g, I.nn_initial_params(seed + 501))
    kw = dict(sloppy_prec=hisq.HISQ_HALF, reliable_delta=0.1, evecs=ev32, evals=eps,
              tol_restart=1e-3)
    losses = []
    t_pairs = t_train = 0.0
    made = 0
    k = 0
    while made < n_pairs:
        m = min(nrhs, n_pairs - made)
        t0 = time.perf_counter()
        ee, eo = device_sources(g, m, seed + 1000 + k, two_m)
        b = torch.empty_like(ee)
        hisq.hisq_prepare_source(g, two_m, ee, eo, b)
        del ee, eo
        xd = torch.empty_like(b)
        hisq.hisq_deflate(g, ev32, eps, two_m, b, xd)
        xs = xd.clone()
        hisq.hisq_cg_solve(g, two_m, b, xs, tol=1e-12, **kw)
        Ax = torch.empty_like(b)
        hisq.hisq_mdagm(g, two_m, xd, Ax)
        R, E = b - Ax, xs - xd
        del b, xd, xs, Ax
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        losses += list(hisq.hisq_nn_train(net, R, E, batch=min(batch, m), steps=steps_per_batch,
                                          lr=lr, flags=hisq.HISQ_NN_NORMALIZE))
        torch.cuda.synchronize()
        t_pairs += t1 - t0
        t_train += time.perf_counter() - t1
        del R, E
        made += m
        k += 1
    say(f"learned guess: {made} pairs streamed ({t_pairs:.1f} s of solves), "
        f"{len(losses)} Adam steps ({t_train:.1f} s), loss {losses[0]:.3f} -> "
        f"{np.mean(losses[-20:]):.3f}")
    return net, {"training_pairs": made, "pairs_seconds": t_pairs, "train_steps": len(losses),
                 "batch": batch, "train_seconds": t_train, "loss_first": float(losses[0]),
                 "loss_last20_mean": float(np.mean(losses[-20:])),
                 "streamed": f"{nrhs} pairs at a time, trained on and dropped"}


def to_full(soa, dims, parity):
    """[3][Vh] parity vector (numpy) -> full lattice [T][Z][Y][X][3], zeros elsewhere."""
    X, Y, Z, T = dims
    V = X * Y * Z * T
    lex = np.arange(V, dtype=np.int64)
    x = lex % X
    y = (lex // X) % Y
    z = (lex // (X * Y)) % Z
    t = lex // (X * Y * Z)
    sel = lex[((x + y + z + t) % 2) == parity]
    flat = np.zeros((V, 3), dtype=np.complex128)
    flat[sel, :] = soa[:, sel >> 1].T
    return flat.reshape(T, Z, Y, X, 3)


def oracle_residuals(F, L, dims, two_m, y_soa, x_soa):
    """||y - A x|| / ||y|| evaluated by the oracle (FP64, its own stencil);
    called from the cpu_baseline leg only."""
    from oracle import hisq_oracle as O
    out = []
    for j in range(y_soa.shape[0]):
        ye = to_full(y_soa[j], dims, 0)
        xe = to_full(x_soa[j], dims, 0)
        out.append(O.norm(ye - O.apply_A(F, L, two_m, xe)) / O.norm(ye))
    return out


def cpu_baseline(W, N, cfg, y_soa, x_soa, n_ev, iters):
    """The oracle on the host cores (the only place this script runs it): a
    bounded sample of the headline workload timed - one source's
    preparation, 4 of the n_ev deflation vectors (scaled to n_ev), 3 CG
    iterations (scaled to the iteration count of the FP64 deflated solve,
    which the oracle's own CG matches to 1%), odd reconstruction - and, with
    the same host links, the oracle's FP64 true residual of the GPU's mixed
    solutions of the given sources."""
    from oracle import hisq_oracle as O
    from paper_2502_00152_amd import inputs as I
    dims, two_m = cfg["dims"], cfg["two_m"]
    t0 = time.perf_counter()
    F, L = O.fold_links(W.cpu().numpy(), N.cpu().numpy(), cfg["c_fat"], cfg["c_long"])
    t_fold = time.perf_counter() - t0
    checks = oracle_residuals(F, L, dims, two_m, y_soa, x_soa)
    eta = to_full(y_soa[0], dims, 0)  # any full-lattice field of the right shape
    t0 = time.perf_counter()
    y = O.source_even(F, L, two_m, eta)
    t_src = time.perf_counter() - t0
    n = 3 * int(np.prod(dims)) // 2
    k_s = 4
    Vs = I.gaussian_even_vectors(k_s, n, 77).T
    yc = O.to_compact(y, dims)
    t0 = time.perf_counter()
    x0c = O.deflation_guess(Vs, np.linspace(0.01, 1.0, k_s), yc)
    t_defl = (time.perf_counter() - t0) * n_ev / k_s
    n_it = 3
    t0 = time.perf_counter()
    O.solve_even(F, L, two_m, y, x0=O.from_compact(x0c, dims), tol=1e-30, max_iter=n_it)
    t_cg = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.reconstruct_odd(F, L, two_m, y, eta)
    t_rec = time.perf_counter() - t0
    per_solve = t_src + t_defl + t_cg / n_it * iters + t_rec
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": O.n_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "oracle_true_residual_of_gpu_solutions": checks,
            "link_fold_seconds": t_fold,
            "sample": (f"one source of the 48^3x96 workload on the host: oracle source "
                       f"preparation ({t_src:.1f} s), the deflation projection with {k_s} of "
                       f"{n_ev} vectors scaled to {n_ev} ({t_defl:.1f} s), {n_it} oracle CG "
                       f"iterations ({t_cg:.1f} s) scaled to the {iters} iterations of the FP64 "
                       f"deflated solve, odd reconstruction ({t_rec:.1f} s); extrapolated")}


def stencil_roofline(prof, vh, nrhs):
    """Live roofline of the CG's 16-bit half stencil from the sampled HIP events."""
    n_plain, ms_plain = prof["dslash_h16"]
    n_aux, ms_aux = prof["dslash_h16_aux"]
    bytes_total = (n_plain * dslash_alg_bytes(vh, nrhs, 0, 4, 2, 16)
                   + n_aux * dslash_alg_bytes(vh, nrhs, 1, 4, 2, 16))
    launches = n_plain + n_aux
    if not launches:
        return None
    avg_ms = (ms_plain + ms_aux) / launches
    bpl = bytes_total / launches
    achieved = bpl / avg_ms / 1e6  # GB/s
    ops = STENCIL_FLOPS_PER_SITE_RHS * nrhs * vh
    return {"bound": "hbm",
            "kernel": f"k_dslash<float, h16p, q16s> (half stencil, packed 16-bit vectors "
                      f"and links, int16 dot products, FP32 accumulation, {nrhs} RHS)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "launches_timed": launches, "timed_every": PROFILE_PERIOD,
            "avg_launch_us": avg_ms * 1e3, "alg_bytes_per_launch": bpl,
            "ops_per_launch": ops, "arith_intensity_op_per_byte": ops / bpl,
            "alu_achieved_Tops": ops / avg_ms / 1e9, "alu_peak_Tops": DOT2_VALU_PEAK_TOPS,
            "alu_frac": ops / avg_ms / 1e9 / DOT2_VALU_PEAK_TOPS,
            "peak_note": ("algorithmic bytes per launch / average launch time (HIP events on "
                          "the launch stream, every 16th launch) against 8 TB/s; ops = the "
                          "1146 flops per site and RHS, here as int16 dot products (157.3 T "
                          "ops/s, ridge 19.7 op/B)")}


PROFILE_CLASSES = ("dslash", "dslash_aux", "dslash_aux2", "dslash_f32", "dslash_f32_aux",
                   "dslash_f32_aux2", "dslash_q16", "dslash_q16_aux", "dslash_h16",
                   "dslash_h16_aux", "blas", "gemm", "nn_layer")


def projection_rate(sample, k, n, N):
    """MFMA rate of the deflation projection launches in the timed steps
    (V^H B and V C: 8 k n N flops each, FP32 vectors widened onto the FP64
    matrix cores at this shape), from the sampled HIP-event times."""
    if not sample or not sample[0]:
        return None
    avg_ms = sample[1] / sample[0]
    tflops = 8.0 * k * n * N / (avg_ms * 1e-3) / 1e12
    return {"k": k, "n": n, "launches_timed": sample[0], "avg_us": avg_ms * 1e3,
            "mfma_tflops": tflops, "peak_tflops": FP64_MFMA_PEAK_TFLOPS,
            "frac_of_fp64_mfma_peak": tflops / FP64_MFMA_PEAK_TFLOPS,
            "note": ("V^H B and V C launches timed by HIP events; hardware MFMA counters "
                     "of the same kernels: profiles/gemm_projection_32x32x32x64.md")}


def headline(args, out):
    """The 48^3 x 96 learned + mixed + batched step."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    cfg = I.workload(4)
    dims, two_m, tol, n_ev, nrhs = cfg["dims"], cfg["two_m"], cfg["tol"], cfg["n_ev"], cfg["nrhs"]
    if args.n_ev:
        n_ev = args.n_ev
    say(f"setup {cfg['name']}")
    g, W, N, t_pack = device_gauge(cfg)
    ee, eo = device_sources(g, nrhs, cfg["seed_src"][0], two_m)
    evecs, lam, eig = eigensolve(g, two_m, n_ev, args.eig_tol, cfg["seed_eig"], "48^3x96",
                                 args.eig_block)
    eps = lam - two_m * two_m
    ev32 = torch.empty(evecs.shape, dtype=torch.complex64, device="cuda")
    hisq.hisq_convert_vectors(evecs, ev32)  # single-precision eigenvectors (section 3)
    net, learn = train_streamed(g, ev32, eps, two_m, args.pairs, nrhs, cfg["seed_eig"],
                                args.train_steps_per_batch)
    y = torch.empty_like(ee)
    x = torch.empty_like(ee)
    po = torch.empty_like(eo)
    kept = []
    kw = dict(sloppy_prec=hisq.HISQ_HALF, reliable_delta=0.1, evecs=ev32, evals=eps,
              tol_restart=1e-3)

    def step(with_guess=True):
        hisq.hisq_prepare_source(g, two_m, ee, eo, y)
        hisq.hisq_deflate(g, ev32, eps, two_m, y, x)
        if with_guess:
            kept[:] = hisq.hisq_nn_guess(net, two_m, y, x,
                                         flags=hisq.HISQ_NN_NORMALIZE | hisq.HISQ_NN_BF16,
                                         evecs=ev32, evals=eps)
        res = hisq.hisq_cg_solve(g, two_m, y, x, tol=tol, **kw)
        hisq.hisq_reconstruct_odd(g, two_m, x, eo, po)
        return res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    hisq.hisq_profile_enable(True, PROFILE_PERIOD)
    for cls in PROFILE_CLASSES:
        hisq.hisq_profile_read(cls)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    hisq.hisq_profile_enable(False)
    prof = {cls: hisq.hisq_profile_read(cls) for cls in PROFILE_CLASSES}
    last = results[-1]
    assert all(all(r.converged) for r in results), "a timed solve did not converge"
    value = nrhs * args.steps / t_steps
    say(f"{args.steps} steps in {t_steps:.2f} s: {value:.2f} solves/s, iterations "
        f"{min(last.iterations)}-{max(last.iterations)}, guess kept for {sum(kept)} of {nrhs}")
    roof = stencil_roofline(prof, g.vh, nrhs)
    if roof:
        roof["traffic"] = read_traffic("dslash_h16_traffic_48x48x48x96.md")
        say(f"16-bit stencil: {roof['avg_launch_us']:.0f} us per launch, "
            f"{roof['achieved']:.0f} GB/s ({roof['frac']:.3f} of peak)")
    x_mixed = x.clone()

    # the same step without the learned guess
    step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rn = step(False)
    torch.cuda.synchronize()
    t_no = time.perf_counter() - t0
    without = {"solves_per_s": nrhs / t_no, "mean_iterations": float(np.mean(rn.iterations)),
               "max_true_residual": max(rn.true_residual)}
    say(f"without the guess: {nrhs / t_no:.2f} solves/s, mean iterations "
        f"{np.mean(rn.iterations):.1f} (with: {np.mean(last.iterations):.1f})")
    net.close()

    # when the reliable update is taken (paper section 3: at the delta_rd
    # trigger): the RHS stops at its trigger until the next host poll (the
    # default for 16-bit vectors), goes on iterating until the poll, or the
    # host polls after every iteration
    ru_variants = {}
    if not args.no_ru_variants:
        for name, freeze, interval in (("stop_at_trigger_poll_16", 1, 16),
                                       ("run_on_to_poll_16", 0, 16),
                                       ("poll_every_iteration", 0, 1)):
            hisq.hisq_set_tuning("cg_reliable_freeze", freeze)
            try:
                hisq.hisq_prepare_source(g, two_m, ee, eo, y)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                hisq.hisq_deflate(g, ev32, eps, two_m, y, x)
                rv = hisq.hisq_cg_solve(g, two_m, y, x, tol=tol, check_interval=interval, **kw)
                hisq.hisq_reconstruct_odd(g, two_m, x, eo, po)
                torch.cuda.synchronize()
                tv = time.perf_counter() - t0
            finally:
                hisq.hisq_set_tuning("cg_reliable_freeze", -1)
            ru_variants[name] = {"solves_per_s": nrhs / tv,
                                 "mean_iterations": float(np.mean(rv.iterations)),
                                 "mean_reliable_updates": float(np.mean(rv.reliable_updates)),
                                 "max_true_residual": max(rv.true_residual)}
            say(f"reliable updates, {name}: {nrhs / tv:.2f} solves/s, mean iterations "
                f"{np.mean(rv.iterations):.1f}, {np.mean(rv.reliable_updates):.1f} updates")

    # FP64 throughout (FP64 eigenvectors, single deflation, FP64 CG), once
    hisq.hisq_prepare_source(g, two_m, ee, eo, y)
    x64 = torch.empty_like(y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hisq.hisq_deflate(g, evecs, eps, two_m, y, x64)
    r64 = hisq.hisq_cg_solve(g, two_m, y, x64, tol=tol)
    hisq.hisq_reconstruct_odd(g, two_m, x64, eo, po)
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    diff = ((x_mixed - x64).abs().pow(2).sum(dim=(1, 2)).sqrt()
            / x64.abs().pow(2).sum(dim=(1, 2)).sqrt()).cpu().numpy()
    fp64 = {"solves_per_s": nrhs / t_fp64, "mean_iterations": float(np.mean(r64.iterations)),
            "max_true_residual": max(r64.true_residual),
            "path": "FP64 eigenvectors, single deflation, FP64 CG"}
    say(f"FP64 deflated: {fp64['solves_per_s']:.2f} solves/s, mean iterations "
        f"{fp64['mean_iterations']:.1f}; mixed vs FP64 solutions: max relative difference "
        f"{diff.max():.2e}")
    del evecs
    torch.cuda.empty_cache()

    # plain FP64 even-odd CG, no deflation, one source
    xs = torch.zeros((1, 3, g.vh), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp = hisq.hisq_cg_solve(g, two_m, y[:1].clone(), xs, tol=tol)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain = {"solves_per_s": 1.0 / t_plain, "iterations": rp.iterations[0], "seconds": t_plain,
             "sources": 1}
    say(f"plain FP64 CG: {t_plain:.2f} s, {rp.iterations[0]} iterations")

    # per-solve error: each mixed solution's distance from the FP64 path's,
    # with its bound (||r|| + ||r'||) ||y|| / lambda_1, the FP64 true residuals
    # the library reports, and (cpu_baseline leg) the oracle's FP64 true
    # residual of sources 0 and 1
    ynorm = y.abs().pow(2).sum(dim=(1, 2)).sqrt().cpu().numpy()
    xnorm = x64.abs().pow(2).sum(dim=(1, 2)).sqrt().cpu().numpy()
    bound = [(last.true_residual[j] + r64.true_residual[j]) * ynorm[j] / lam[0] / xnorm[j]
             for j in range(nrhs)]
    per_solve = {"reported_true_residual": list(last.true_residual),
                 "rel_diff_vs_fp64_solution": diff.tolist(),
                 "rel_diff_bound": bound,
                 "oracle_true_residual_sources_0_1": None}
    cpu = None
    if not args.no_cpu_baseline:
        ys = y[:2].cpu().numpy()
        xm = x_mixed[:2].cpu().numpy()
        cpu = cpu_baseline(W, N, cfg, ys, xm, n_ev, int(round(np.mean(r64.iterations))))
        per_solve["oracle_true_residual_sources_0_1"] = cpu["oracle_true_residual_of_gpu_solutions"]
        say(f"oracle on the host: {cpu['value']:.5f} solves/s ({cpu['cores']} threads, "
            f"{cpu['cpu_model']}); oracle residuals of sources 0, 1: "
            f"{cpu['oracle_true_residual_of_gpu_solutions']}")
    del W, N
    g_vh = g.vh
    g.close()

    out.update({
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_steps / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("int16 fixed-point links, search direction and A p (norm per site) with "
                  "int16 dot products and FP32 accumulation; FP32 residual and correction; "
                  "FP64 reductions, reliable updates, solution and source/reconstruction; "
                  "FP32 eigenvectors with FP64 projection coefficients; BF16 network weights "
                  "with FP32 arithmetic"),
        "data": "synthetic",
        "config": {"workload": cfg["name"], "lattice": "x".join(map(str, dims)),
                   "eps": cfg["eps"], "two_m": two_m, "sources_per_step": nrhs,
                   "n_ev": n_ev, "n_ev_config": 512, "training_pairs": learn["training_pairs"],
                   "training_pairs_config": 2000, "tol": tol,
                   "path": ("deflation with FP32 eigenvectors, learned correction (BF16 "
                            "weights, projected off the deflation space, kept per source where "
                            "it lowers the FP64 residual), batched mixed-precision CG (16-bit "
                            "sloppy operator and search direction, FP64 reliable updates at "
                            "delta_rd 0.1), re-deflation at delta_tr 1e-3"),
                   "reduced": (f"{n_ev} eigenpairs and {learn['training_pairs']} streamed "
                               "training pairs instead of 512 and 2000, to keep the run within "
                               "minutes (a 512-pair eigensolve at this volume takes far longer "
                               "than the run; its memory fits: one FP64 basis of n_kr + block "
                               "vectors)")},
        "roofline": roof,
        "cpu_baseline": cpu,
        "iterations_per_source": last.iterations,
        "reliable_updates_per_source": last.reliable_updates,
        "redeflations_per_source": last.redeflations,
        "max_true_residual": max(max(r.true_residual) for r in results),
        "per_solve_error": per_solve,
        "learned_guess": dict(learn, kept=list(kept), without_guess=without),
        "reliable_update_timing": ru_variants,
        "deflated_fp64_cg": fp64,
        "plain_fp64_cg": plain,
        "speedup_vs_plain_fp64_cg": value / plain["solves_per_s"],
        "eigensolve": eig,
        "gauge_pack_seconds": t_pack,
        "kernel_sample": {k: {"launches_timed": v[0],
                              "avg_us": v[1] / v[0] * 1e3 if v[0] else None}
                          for k, v in prof.items()},
        "projection": projection_rate(prof.get("gemm"), n_ev, nrhs, 3 * g_vh),
    })


def secondary_16(args):
    """The 16^3 x 32 deflated workload (eps 0.5, 2m = 0.01, 12 sources, 64
    eigenpairs): the mixed step, FP64 throughout and plain CG."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    cfg = I.workload(1)
    two_m, tol, nrhs, n_ev = cfg["two_m"], cfg["tol"], cfg["nrhs"], cfg["n_ev"]
    dims = cfg["dims"]
    W = torch.from_numpy(I.random_su3_field(dims, cfg["eps"], cfg["seed_fat"])).cuda()
    N = torch.from_numpy(I.random_su3_field(dims, cfg["eps"], cfg["seed_long"])).cuda()
    g = hisq.Gauge(dims, W, N, cfg["c_fat"], cfg["c_long"])
    del W, N
    eta = np.stack([I.gaussian_source(dims, sd) for sd in cfg["seed_src"]])
    ee = torch.empty((nrhs, 3, g.vh), dtype=torch.complex128, device="cuda")
    eo = torch.empty_like(ee)
    hisq.hisq_spinor_split(g, torch.from_numpy(eta).cuda(), ee, eo)
    evecs, lam, eig = eigensolve(g, two_m, n_ev, tol, cfg["seed_eig"], "16^3x32")
    eps = lam - two_m * two_m
    ev32 = torch.empty(evecs.shape, dtype=torch.complex64, device="cuda")
    hisq.hisq_convert_vectors(evecs, ev32)
    y = torch.empty_like(ee)
    x = torch.empty_like(ee)
    po = torch.empty_like(eo)

    def step_mixed():
        hisq.hisq_prepare_source(g, two_m, ee, eo, y)
        hisq.hisq_deflate(g, ev32, eps, two_m, y, x)
        r = hisq.hisq_cg_solve(g, two_m, y, x, tol=tol, sloppy_prec=hisq.HISQ_HALF,
                               reliable_delta=0.1, evecs=ev32, evals=eps, tol_restart=1e-3)
        hisq.hisq_reconstruct_odd(g, two_m, x, eo, po)
        return r

    def step_fp64():
        hisq.hisq_prepare_source(g, two_m, ee, eo, y)
        hisq.hisq_deflate(g, evecs, eps, two_m, y, x)
        r = hisq.hisq_cg_solve(g, two_m, y, x, tol=tol)
        hisq.hisq_reconstruct_odd(g, two_m, x, eo, po)
        return r

    res = {}
    for name, fn in (("mixed", step_mixed), ("fp64", step_fp64)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            r = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert all(r.converged)
        res[name] = {"solves_per_s": nrhs * 5 / dt, "mean_iterations": float(np.mean(r.iterations)),
                     "max_true_residual": max(r.true_residual)}
    xs = torch.zeros((1, 3, g.vh), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp = hisq.hisq_cg_solve(g, two_m, y[:1].clone(), xs, tol=tol)
    torch.cuda.synchronize()
    res["plain_fp64_cg"] = {"solves_per_s": 1.0 / (time.perf_counter() - t0),
                            "iterations": rp.iterations[0]}
    res["eigensolve"] = eig
    res["speedup_mixed_vs_plain"] = res["mixed"]["solves_per_s"] / res["plain_fp64_cg"]["solves_per_s"]
    say(f"16^3x32: mixed {res['mixed']['solves_per_s']:.1f} solves/s, FP64 deflated "
        f"{res['fp64']['solves_per_s']:.1f}, plain {res['plain_fp64_cg']['solves_per_s']:.1f}")
    g.close()
    return res


def uneven_leg():
    """The uneven batch: 8^4 (32 RHS), 12^4 (16), 16^3 x 32 (8), 24^3 x 48 (4),
    each at 2m = 0.1, 0.02, 0.005 (the masses of a lattice in one batched solve),
    the four systems solved together (every RHS is checked against the oracle
    in tests/test_gpu_uneven_batch.py)."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    B = I.UNEVEN_BATCH
    lat = []
    for l, (dims, nrhs) in enumerate(B["lattices"]):
        Wd = I.random_su3_field_device(dims, B["eps"], 30000 + 1000 * l + 1)
        Nd = I.random_su3_field_device(dims, B["eps"], 30000 + 1000 * l + 2)
        g = hisq.Gauge(dims, Wd, Nd, I.C_FAT, I.C_LONG)
        bs = []
        for k in range(len(B["masses"])):
            gen = torch.Generator(device="cuda")
            gen.manual_seed(30000 + 1000 * l + 100 + 10 * k)
            bs.append(torch.randn((nrhs, 3, g.vh), dtype=torch.complex128, device="cuda",
                                  generator=gen))
        del Wd, Nd
        lat.append(dict(dims=dims, g=g, b=torch.cat(bs), masses=np.repeat(B["masses"], nrhs)))
    out = {}
    # one stream per system, or every chunk of iterations of the four systems
    # as one captured graph (bitwise the same solutions)
    for mode, tag in ((0, ""), (1, "_one_graph")):
        hisq.hisq_set_tuning("cg_multi_graph", mode)
        try:
            for name, sp in (("fp64", hisq.HISQ_FP64), ("half", hisq.HISQ_HALF)):
                systems = [(d["g"], d["masses"], d["b"], torch.zeros_like(d["b"])) for d in lat]
                hisq.hisq_cg_solve_multi(systems, tol=B["tol"], sloppy_prec=sp)  # warm
                systems = [(d["g"], d["masses"], d["b"], torch.zeros_like(d["b"])) for d in lat]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = hisq.hisq_cg_solve_multi(systems, tol=B["tol"], sloppy_prec=sp)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                n = sum(d["b"].shape[0] for d in lat)
                o = {"solves_per_s": n / dt, "solves": n, "seconds": dt,
                     "max_iterations_per_system": [max(r.iterations) for r in res],
                     "max_true_residual_per_system": [max(r.true_residual) for r in res],
                     "all_converged": all(all(r.converged) for r in res)}
                out[name + tag] = o
        finally:
            hisq.hisq_set_tuning("cg_multi_graph", -1)
    for d in lat:
        d["g"].close()
    say(f"uneven batch: {out['half']['solves_per_s']:.0f} solves/s (16-bit sloppy), "
        f"{out['fp64']['solves_per_s']:.0f} (FP64); one graph per chunk: "
        f"{out['half_one_graph']['solves_per_s']:.0f}, {out['fp64_one_graph']['solves_per_s']:.0f}")
    return out


def dslash_scan(reps=10):
    """Half-stencil launch times beyond the last-level cache: 32^3 x 64 and
    48^3 x 96, 1, 12 and 24 RHS, FP64, FP32 (FP32 links) and the CG's 16-bit
    form (16-bit vectors and links, at the boundary FP32 vectors: the call
    includes the conversions, so kernel_us comes from the profile sample)."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    out = {}
    for dims in ((32, 32, 32, 64), (48, 48, 48, 96)):
        W = I.random_su3_field_device(dims, 0.5, 20001)
        N = I.random_su3_field_device(dims, 0.5, 20002)
        g = hisq.Gauge(dims, W, N, I.C_FAT, I.C_LONG)
        del W, N
        torch.cuda.empty_cache()
        key = "x".join(map(str, dims))
        out[key] = {}
        for name, dt, prec, rb, lb, sb, cls in (
                ("f64", torch.complex128, hisq.HISQ_FP64, 8, 8, 48, "dslash"),
                ("f32", torch.complex64, hisq.HISQ_FP32, 4, 4, 24, "dslash_f32"),
                ("h16", torch.complex64, hisq.HISQ_HALF, 4, 2, 16, "dslash_h16")):
            for nrhs in (1, 12, 24):
                if name == "f64" and dims[0] == 48 and nrhs == 24:
                    continue
                a = torch.randn((nrhs, 3, g.vh), dtype=dt, device="cuda")
                b = torch.empty_like(a)
                for _ in range(2):
                    hisq.hisq_dslash_eo(g, 0, a, b, prec=prec)
                torch.cuda.synchronize()
                hisq.hisq_profile_enable(True, 1)
                hisq.hisq_profile_read(cls)
                for _ in range(reps):
                    hisq.hisq_dslash_eo(g, 0, a, b, prec=prec)
                torch.cuda.synchronize()
                hisq.hisq_profile_enable(False)
                n, ms = hisq.hisq_profile_read(cls)
                us = ms / max(n, 1) * 1e3
                alg = dslash_alg_bytes(g.vh, nrhs, 0, rb, lb, sb)
                out[key][f"{name}_{nrhs}rhs"] = {"kernel_us": us, "algorithmic_bytes": alg,
                                                  "GB_s": alg / us / 1e3,
                                                  "frac_of_hbm_peak": alg / us / 1e3 / HBM_PEAK_GBS}
                del a, b
        g.close()
        torch.cuda.empty_cache()
    say("dslash scan: " + ", ".join(f"{k} {v['h16_12rhs']['frac_of_hbm_peak']:.2f} (h16 12 RHS) "
                                     f"{v['f64_1rhs']['frac_of_hbm_peak']:.2f} (f64 1 RHS)"
                                     for k, v in out.items()))
    return out


def pmc_probe(which):
    """Short run for hardware-counter passes: a few launches of the CG's
    16-bit half stencil with 12 RHS at the workload's volume (48: 48^3 x 96,
    16: 16^3 x 32), or (32) the half stencil with 24 RHS at 32^3 x 64 in
    16-bit, FP32 and FP64 storage; then a plain 1 GiB copy whose counter
    readings calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    cfg = I.workload({"48": 4, "16": 1, "32": 2}[which])
    g, W, N, _ = device_gauge(cfg)
    del W, N
    torch.cuda.empty_cache()
    if which == "32":
        for prec, dt in ((hisq.HISQ_HALF, torch.complex64), (hisq.HISQ_FP32, torch.complex64),
                         (hisq.HISQ_FP64, torch.complex128)):
            x = torch.randn((24, 3, g.vh), dtype=dt, device="cuda")
            y = torch.empty_like(x)
            for _ in range(3):
                hisq.hisq_dslash_eo(g, 0, x, y, prec=prec)
            del x, y
            torch.cuda.empty_cache()
    else:
        x = torch.randn((12, 3, g.vh), dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            hisq.hisq_dslash_eo(g, 0, x, y, prec=hisq.HISQ_HALF)
            hisq.hisq_mdagm(g, cfg["two_m"], x, y, prec=hisq.HISQ_HALF)
        del x, y
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    g.close()
    print(json.dumps({"pmc_probe": which, "copy_bytes": a.numel() * 8,
                      "kernel_source_hash": kernel_source_hash()}), flush=True)


def gemm_probe():
    """The deflation projection (Eq. (4)) at 32^3 x 64 with FP32 eigenvectors:
    64 vectors x 12 RHS and 256 x 24, with FP64 arithmetic and on the FP32
    matrix cores, five calls each (for kernel traces and MFMA counters)."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    cfg = I.workload(2)
    g, W, N, _ = device_gauge(cfg)
    del W, N
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    out = {}
    for k, n in ((64, 12), (256, 24)):
        V = torch.randn((k, 3, g.vh), dtype=torch.complex64, device="cuda", generator=gen)
        B = torch.randn((n, 3, g.vh), dtype=torch.complex128, device="cuda", generator=gen)
        x = torch.empty_like(B)
        eps = np.linspace(1e-3, 0.2, k)
        for mode in (0, 1):
            hisq.hisq_set_tuning("gemm_fp32_mfma", mode)
            try:
                hisq.hisq_deflate(g, V, eps, cfg["two_m"], B, x)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(5):
                    hisq.hisq_deflate(g, V, eps, cfg["two_m"], B, x)
                torch.cuda.synchronize()
                out[f"{k}x{n}_fp32_mfma_{mode}_ms"] = (time.perf_counter() - t0) / 5 * 1e3
            finally:
                hisq.hisq_set_tuning("gemm_fp32_mfma", -1)
        del V, B, x
        torch.cuda.empty_cache()
    g.close()
    print(json.dumps({"gemm_probe": out}), flush=True)


def eig_recipe(n_ev=512, n_kr=640, block=6):
    """The learned-guess lattice with its recipe's 512 eigenpairs, run on its
    own (the eigensolve takes longer than a benchmark run): the block
    eigensolve with FP32 output (one FP64 basis of n_kr + block vectors, about
    190 GB with its work blocks, besides 65 GB of FP32 eigenvectors), then two
    deflated, re-deflated mixed-precision solves of 12 sources with those
    eigenvectors (deflation + CG timed).  Prints one JSON line."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    cfg = I.workload(4)
    two_m = cfg["two_m"]
    g, W, N, _ = device_gauge(cfg)
    del W, N
    torch.cuda.empty_cache()
    say(f"gauge ready, {torch.cuda.mem_get_info()[0] / 1e9:.1f} GB free")
    ev = torch.empty((n_ev, 3, g.vh), dtype=torch.complex64, device="cuda")
    last = [0.0]

    def prog(r, j, mv, sec):
        if sec - last[0] >= 30.0:
            last[0] = sec
            say(f"eigensolve restart {r} step {j} matvecs {mv} {sec:.0f} s")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, lam, es = hisq.hisq_eigensolve(g, two_m, n_ev, ev, n_kr=n_kr, tol=1e-10,
                                      seed=cfg["seed_eig"], block=block, progress=prog)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    say(f"eigensolve {t_eig:.1f} s, {es.matvecs} matvecs, {es.restarts} restarts, "
        f"max residual {es.max_residual:.2e}")
    eps = lam - two_m * two_m
    solves = []
    for _ in range(2):
        ee, eo = device_sources(g, 12, cfg["seed_src"][0], two_m)
        y = torch.empty_like(ee)
        hisq.hisq_prepare_source(g, two_m, ee, eo, y)
        del ee, eo
        x = torch.empty_like(y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hisq.hisq_deflate(g, ev, eps, two_m, y, x)
        r = hisq.hisq_cg_solve(g, two_m, y, x, tol=cfg["tol"], sloppy_prec=hisq.HISQ_HALF,
                               reliable_delta=0.1, evecs=ev, evals=eps, tol_restart=1e-3)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        solves.append({"seconds": dt, "solves_per_s": 12 / dt, "iterations": r.iterations,
                       "max_true_residual": max(r.true_residual),
                       "converged": all(r.converged)})
        say(f"deflation + mixed CG of 12 sources: {dt:.2f} s ({12 / dt:.2f} solves/s), "
            f"iterations {min(r.iterations)}-{max(r.iterations)}")
        del y, x
    g.close()
    print(json.dumps({"workload": cfg["name"], "n_ev": n_ev, "n_kr": n_kr, "block": block,
                      "eigensolve": {"seconds": t_eig, "matvecs": es.matvecs,
                                     "restarts": es.restarts, "cheb_degree": es.cheb_degree,
                                     "max_residual": es.max_residual,
                                     "lambda_1": float(lam[0]), "lambda_last": float(lam[-1])},
                      "solves": solves}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="skip the legs after the headline once the run has used this long")
    ap.add_argument("--eig-tol", type=float, default=1e-10)
    ap.add_argument("--eig-block", type=int, default=6,
                    help="Lanczos block size of the 48^3 x 96 eigensolve (0: one vector per step)")
    ap.add_argument("--pairs", type=int, default=48, help="training pairs for the learned guess")
    ap.add_argument("--n-ev", type=int, default=0,
                    help="eigenpairs of the headline workload (0: the workload's 128)")
    ap.add_argument("--train-steps-per-batch", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-dslash-scan", action="store_true")
    ap.add_argument("--no-ru-variants", action="store_true",
                    help="skip the reliable-update timing variants of the headline solve")
    ap.add_argument("--pmc-probe", choices=("48", "16", "32"))
    ap.add_argument("--gemm-probe", action="store_true",
                    help="time the deflation projection at 32^3 x 64 (for profiles) and exit")
    ap.add_argument("--eig-recipe", action="store_true",
                    help="512 eigenpairs at 48^3 x 96 and two deflated solves with them "
                         "(about 12 minutes), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); run with --gpus 1", flush=True)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", flush=True)
        sys.exit(1)
    if args.pmc_probe:
        pmc_probe(args.pmc_probe)
        return
    if args.gemm_probe:
        gemm_probe()
        return
    if args.eig_recipe:
        eig_recipe()
        return
    out = {}
    headline(args, out)
    legs = {}
    for name, skip, fn in (("deflated_cg_16x16x16x32", args.no_secondary, lambda: secondary_16(args)),
                           ("uneven_batch", args.no_uneven, uneven_leg),
                           ("dslash_scan", args.no_dslash_scan, dslash_scan)):
        if skip:
            continue
        if time.perf_counter() - T0 > args.budget_s:
            legs[name] = {"skipped": f"run time budget of {args.budget_s:.0f} s used"}
            say(f"skipping {name}: budget used")
            continue
        legs[name] = fn()
    out.update(legs)
    out["bench_seconds"] = time.perf_counter() - T0
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
