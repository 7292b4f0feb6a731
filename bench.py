"""Benchmark of the HISQ deflated even-odd CG path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-dslash-scan] [--no-plain-cg] [--pmc-probe]

Workload (the deflated-CG configuration, synthetic): 16^3 x 32 lattice, random
SU(3) fat and long links (eps 0.5, long links scaled by -1/24, staggered phases
and antiperiodic time folded in), 2m = 0.01, 12 Gaussian sources, 64 lowest
eigenpairs, true-residual target 1e-10 (FP64 residual b - A x).

One step solves the 12 sources end to end on the GPU, inputs already resident
in HBM, with the paper's production method (sections 2 and 3): source
preparation y_e = 2m eta_e - D_eo eta_o (FP64); deflation guess
x0 = V diag(1/lambda) V^H y_e with single-precision eigenvectors; batched
mixed-precision CG (16-bit fixed-point links, search direction and A p
with a norm per site, FP32 residual and correction, FP64 dot products, FP64
reliable updates at delta_rd = 0.1) with re-deflation whenever the true
residual has fallen by delta_tr = 1e-3 since the last deflation, to
||y - A x|| <= 1e-10 ||y||; odd reconstruction psi_o = (eta_o - D_oe psi_e) / (2m)
(FP64).  Setup (gauge packing) and the eigensolve (FP64) are outside the
timed region, as in the paper, which amortises the eigensolve over the solves
of one gauge field; both are timed and reported.
value = solves per second = 12 * K / (time of K steps).

Also reported: the same step in FP64 throughout (FP64 eigenvectors, single
deflation, FP64 CG), plain FP64 even-odd CG (no deflation, one source at a
time), the relative difference of the mixed solutions from the FP64 ones, the
half-stencil bandwidth at 32^3 x 64 (beyond the 256 MB last-level cache) in
FP64, FP32 and BF16, the roofline of the CG's 16-bit half stencil measured
live with HIP events inside the timed region, and the oracle timed on the
host cores.
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
STENCIL_FLOPS_PER_SITE_RHS = 16 * 66 + 15 * 6  # 16 SU(3) x vector products and their sum
PROFILE_PERIOD = 16
LEARNED_PAIRS = 128   # training pairs the solver generates for the learned guess
LEARNED_STEPS = 400   # Adam steps, mini-batches of 8


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


def read_traffic(name="dslash_h16_traffic_16x16x16x32.md"):
    """HBM traffic per half-stencil launch from the committed counter summary,
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


def build_problem(cfg):
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    dims = cfg["dims"]
    W = torch.from_numpy(I.random_su3_field(dims, cfg["eps"], cfg["seed_fat"])).cuda()
    N = torch.from_numpy(I.random_su3_field(dims, cfg["eps"], cfg["seed_long"])).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = hisq.Gauge(dims, W, N, cfg["c_fat"], cfg["c_long"])
    t_pack = time.perf_counter() - t0
    del W, N
    eta = np.stack([I.gaussian_source(dims, sd) for sd in cfg["seed_src"]])
    full = torch.from_numpy(eta).cuda()
    nrhs = len(cfg["seed_src"])
    ee = torch.empty((nrhs, 3, g.vh), dtype=torch.complex128, device="cuda")
    eo = torch.empty_like(ee)
    hisq.hisq_spinor_split(g, full, ee, eo)
    torch.cuda.synchronize()
    return g, ee, eo, t_pack


def pmc_probe(cfg):
    """Light run for hardware-counter passes: three iterations of the timed CG
    (12 RHS, 16-bit vectors and links), the half-stencil launches of one CG
    iteration with FP32 vectors and 16-bit links, FP32 links, then FP64, and a
    plain 1 GiB copy whose counter readings calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    from paper_2502_00152_amd import hisq
    g, ee, eo, _ = build_problem(cfg)
    y = torch.empty_like(ee)
    hisq.hisq_prepare_source(g, cfg["two_m"], ee, eo, y)
    hisq.hisq_cg_solve(g, cfg["two_m"], y, torch.zeros_like(y), tol=cfg["tol"], max_iter=3,
                       check_interval=3, sloppy_prec=hisq.HISQ_HALF, raise_on_fail=False)
    for a, prec in ((ee.to(torch.complex64), hisq.HISQ_Q16), (ee.to(torch.complex64), hisq.HISQ_FP32),
                    (ee, hisq.HISQ_FP64)):
        t = torch.empty_like(a)
        out = torch.empty_like(a)
        for _ in range(3):
            hisq.hisq_dslash_eo(g, 1, a, t, prec=prec)
            hisq.hisq_mdagm(g, cfg["two_m"], a, out, prec=prec)
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": "done", "copy_bytes": a.numel() * 8,
                      "kernel_source_hash": kernel_source_hash()}), flush=True)


def dslash_scan(dims=(32, 32, 32, 64), reps=20):
    """Half-stencil GB/s at a lattice whose working set exceeds the LLC, one
    RHS, FP64, FP32 and BF16 storage."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    W = I.random_su3_field_device(dims, 0.5, 20001)
    N = I.random_su3_field_device(dims, 0.5, 20002)
    g = hisq.Gauge(dims, W, N, I.C_FAT, I.C_LONG)
    del W, N
    torch.cuda.empty_cache()
    out = {"lattice": "x".join(map(str, dims)), "nrhs": 1}
    for name, dt, rb in (("f64", torch.complex128, 8), ("f32", torch.complex64, 4),
                         ("bf16", torch.bfloat16, 2)):
        shape = (1, 3, g.vh, 2) if dt == torch.bfloat16 else (1, 3, g.vh)
        a = torch.randn(shape, dtype=dt, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            hisq.hisq_dslash_eo(g, 0, a, b)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            hisq.hisq_dslash_eo(g, 0, a, b)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        alg = dslash_alg_bytes(g.vh, 1, 0, rb)
        out[name] = {"us_per_launch": ms * 1e3, "algorithmic_bytes": alg, "GB_s": alg / ms / 1e6,
                     "frac_of_hbm_peak": alg / ms / 1e6 / HBM_PEAK_GBS}
    g.close()
    return out


def cpu_baseline(cfg, golden):
    """The oracle timed on the host: one source of the workload, with the
    deflated iteration count the oracle itself reached (stored golden value)."""
    from oracle import hisq_oracle as O
    from paper_2502_00152_amd import inputs as I
    dims, two_m = cfg["dims"], cfg["two_m"]
    W = I.random_su3_field(dims, cfg["eps"], cfg["seed_fat"])
    N = I.random_su3_field(dims, cfg["eps"], cfg["seed_long"])
    F, L = O.fold_links(W, N, cfg["c_fat"], cfg["c_long"])
    eta = I.gaussian_source(dims, cfg["seed_src"][0])
    t0 = time.perf_counter()
    y = O.source_even(F, L, two_m, eta)
    t_src = time.perf_counter() - t0
    k = cfg["n_ev"]
    n = 3 * int(np.prod(dims)) // 2
    Vs = I.gaussian_even_vectors(k, n, 77).T  # same shape as the eigenvectors
    lam = np.linspace(0.01, 1.0, k)
    yc = O.to_compact(y, dims)
    t0 = time.perf_counter()
    x0c = O.deflation_guess(Vs, lam, yc)
    t_defl = time.perf_counter() - t0
    n_it = 60
    t0 = time.perf_counter()
    O.solve_even(F, L, two_m, y, x0=O.from_compact(x0c, dims), tol=1e-30, max_iter=n_it)
    t_cg = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.reconstruct_odd(F, L, two_m, y, eta)
    t_rec = time.perf_counter() - t0
    iters = golden["cg_iterations_deflated"]
    per_solve = t_src + t_defl + t_cg / n_it * iters + t_rec
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": O.n_threads(),
            "kind": "oracle",
            "sample": (f"one source of the 16^3x32 workload: oracle source preparation, "
                       f"deflation projection ({k} vectors), {n_it} oracle CG iterations "
                       f"({t_cg:.1f} s) scaled to the {iters} iterations the oracle's own "
                       f"deflated solve takes, odd reconstruction")}


def learned_large():
    """The learned guess on one GPU's share of a large lattice (48^3 x 96,
    2m = 0.002): eigensolve, training pairs from the production solver,
    training, then the production step on 12 fresh sources without and with
    the guess.  Prints one JSON line."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    cfg = I.workload(4)
    dims, two_m, tol, n_ev, nrhs = cfg["dims"], cfg["two_m"], cfg["tol"], cfg["n_ev"], cfg["nrhs"]
    t_all = time.perf_counter()
    W = I.random_su3_field_device(dims, cfg["eps"], cfg["seed_fat"])
    N = I.random_su3_field_device(dims, cfg["eps"], cfg["seed_long"])
    g = hisq.Gauge(dims, W, N, cfg["c_fat"], cfg["c_long"])
    del W, N
    torch.cuda.empty_cache()
    print(f"[learned-48] gauge ready {time.perf_counter() - t_all:.1f} s", flush=True)
    evecs = torch.empty((n_ev, 3, g.vh), dtype=torch.complex128, device="cuda")
    last = [0.0]

    def prog(r, j, mv, sec):
        if sec - last[0] >= 10.0:
            last[0] = sec
            print(f"[learned-48] eigensolve restart {r} step {j} matvecs {mv} {sec:.0f} s", flush=True)

    t0 = time.perf_counter()
    st, lam, est = hisq.hisq_eigensolve(g, two_m, n_ev, evecs, tol=tol, seed=cfg["seed_eig"],
                                        progress=prog)
    t_eig = time.perf_counter() - t0
    eps = lam - two_m * two_m
    ev32 = torch.empty(evecs.shape, dtype=torch.complex64, device="cuda")
    hisq.hisq_convert_vectors(evecs, ev32)
    del evecs
    torch.cuda.empty_cache()
    print(f"[learned-48] eigensolve {t_eig:.1f} s, lambda_1 {lam[0]:.4e}, lambda_64 {lam[-1]:.4e}",
          flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(cfg["seed_eig"] + 500)

    def sources(n):
        a = torch.randn((n, 3, g.vh), dtype=torch.complex128, device="cuda", generator=gen)
        c = torch.randn((n, 3, g.vh), dtype=torch.complex128, device="cuda", generator=gen)
        b = torch.empty_like(a)
        hisq.hisq_prepare_source(g, two_m, a, c, b)
        return b

    kw = dict(sloppy_prec=hisq.HISQ_Q16, reliable_delta=0.1, evecs=ev32, evals=eps,
              tol_restart=1e-3)
    R, E = [], []
    t0 = time.perf_counter()
    for k in range(cfg["n_pairs"] // nrhs):
        b = sources(nrhs)
        xd = torch.empty_like(b)
        hisq.hisq_deflate(g, ev32, eps, two_m, b, xd)
        xs = xd.clone()
        hisq.hisq_cg_solve(g, two_m, b, xs, tol=1e-12, **kw)
        Ax = torch.empty_like(b)
        hisq.hisq_mdagm(g, two_m, xd, Ax)
        R.append(b - Ax)
        E.append(xs - xd)
        del b, xd, xs, Ax
        print(f"[learned-48] training pairs {(k + 1) * nrhs}", flush=True)
    R = torch.cat(R)
    E = torch.cat(E)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    net = hisq.Network(g, I.nn_initial_params(cfg["seed_eig"] + 501))
    t0 = time.perf_counter()
    steps = 200
    losses = hisq.hisq_nn_train(net, R, E, batch=2, steps=steps, lr=1e-2,
                                flags=hisq.HISQ_NN_NORMALIZE)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del R, E
    torch.cuda.empty_cache()
    print(f"[learned-48] training {t_train:.1f} s, loss {losses[0]:.3f} -> "
          f"{np.mean(losses[-20:]):.3f}", flush=True)
    b = sources(nrhs)
    x = torch.empty_like(b)

    def step(with_guess):
        hisq.hisq_deflate(g, ev32, eps, two_m, b, x)
        kept = None
        if with_guess:
            kept = hisq.hisq_nn_guess(net, two_m, b, x,
                                      flags=hisq.HISQ_NN_NORMALIZE | hisq.HISQ_NN_BF16,
                                      evecs=ev32, evals=eps)
        r = hisq.hisq_cg_solve(g, two_m, b, x, tol=tol, **kw)
        return r, kept

    out = {}
    for name, wg in (("without", False), ("with", True)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r, kept = step(wg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert all(r.converged), f"a solve {name} the guess did not converge"
        out[name] = {"solves_per_s": nrhs / dt, "mean_iterations": float(np.mean(r.iterations)),
                     "max_true_residual": max(r.true_residual), "kept": kept}
        print(f"[learned-48] {name} the guess: {nrhs / dt:.2f} solves/s, mean iterations "
              f"{np.mean(r.iterations):.1f}", flush=True)
    net.close()
    g.close()
    print(json.dumps({"workload": cfg["name"], "lattice": "x".join(map(str, dims)),
                      "two_m": two_m, "n_ev": n_ev, "training_pairs": cfg["n_pairs"],
                      "train_steps": steps, "batch": 2, "eigensolve_seconds": t_eig,
                      "pairs_seconds": t_pairs, "train_seconds": t_train,
                      "loss_first": float(losses[0]),
                      "loss_last20_mean": float(np.mean(losses[-20:])),
                      "lambda_1": float(lam[0]), "lambda_64": float(lam[-1]),
                      "sloppy_links": "q16", "unit": "solves/s", **out}), flush=True)


def train_learned_guess(g, evecs, eps, two_m, seed):
    """Train the learned guess on pairs the solver generates: r = the residual
    of the deflation guess of a prepared random source, e = the remaining
    error from an FP64 solve to 1e-12.  Returns the network and timings."""
    import torch
    from paper_2502_00152_amd import hisq, inputs as I
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed + 500)
    R, E = [], []
    t0 = time.perf_counter()
    for _ in range(LEARNED_PAIRS // 16):
        a = torch.randn((16, 3, g.vh), dtype=torch.complex128, device="cuda", generator=gen)
        c = torch.randn((16, 3, g.vh), dtype=torch.complex128, device="cuda", generator=gen)
        b = torch.empty_like(a)
        hisq.hisq_prepare_source(g, two_m, a, c, b)
        xd = torch.empty_like(b)
        hisq.hisq_deflate(g, evecs, eps, two_m, b, xd)
        xs = xd.clone()
        hisq.hisq_cg_solve(g, two_m, b, xs, tol=1e-12)
        hisq.hisq_mdagm(g, two_m, xd, a)
        R.append(b - a)
        E.append(xs - xd)
    R = torch.cat(R)
    E = torch.cat(E)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    net = hisq.Network(g, I.nn_initial_params(seed + 501))
    t0 = time.perf_counter()
    losses = hisq.hisq_nn_train(net, R, E, batch=8, steps=LEARNED_STEPS, lr=1e-2,
                                flags=hisq.HISQ_NN_NORMALIZE)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"[bench] learned guess: {LEARNED_PAIRS} pairs in {t_pairs:.2f} s, {LEARNED_STEPS} "
          f"Adam steps in {t_train:.2f} s, loss {losses[0]:.3f} -> {np.mean(losses[-20:]):.3f}",
          flush=True)
    return net, {"training_pairs": LEARNED_PAIRS, "pairs_seconds": t_pairs,
                 "train_steps": LEARNED_STEPS, "batch": 8, "train_seconds": t_train,
                 "loss_first": float(losses[0]), "loss_last20_mean": float(np.mean(losses[-20:]))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dslash-scan", action="store_true")
    ap.add_argument("--no-plain-cg", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true")
    ap.add_argument("--learned-large", action="store_true",
                    help="measure the learned guess at 48^3 x 96 instead (one JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); run with --gpus 1", flush=True)
        sys.exit(2)

    import torch
    from paper_2502_00152_amd import hisq, inputs as I

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", flush=True)
        sys.exit(1)
    cfg = I.workload(1)
    if args.pmc_probe:
        pmc_probe(cfg)
        return
    if args.learned_large:
        learned_large()
        return
    two_m, tol, nrhs, n_ev = cfg["two_m"], cfg["tol"], cfg["nrhs"], cfg["n_ev"]
    print(f"[bench] setup {cfg['name']}", flush=True)
    g, ee, eo, t_pack = build_problem(cfg)

    # eigensolve: amortised over the solves of this gauge field, outside the step
    evecs = torch.empty((n_ev, 3, g.vh), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, lam, est = hisq.hisq_eigensolve(g, two_m, n_ev, evecs, tol=tol, seed=cfg["seed_eig"])
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    eps = lam - two_m * two_m
    print(f"[bench] eigensolve {t_eig:.2f} s, {est.matvecs} matvecs, {est.restarts} restarts, "
          f"max residual {est.max_residual:.2e}", flush=True)

    ev32 = torch.empty(evecs.shape, dtype=torch.complex64, device="cuda")
    hisq.hisq_convert_vectors(evecs, ev32)  # single-precision eigenvectors (section 3)
    y = torch.empty_like(ee)
    x = torch.empty_like(ee)
    po = torch.empty_like(eo)
    F32 = hisq.HISQ_FP32
    SLOPPY = hisq.HISQ_HALF  # 16-bit links, 16-bit p and A p in the sloppy recurrence

    # learned initial guess (an extension beyond the paper), trained like the
    # eigensolve once per gauge field, outside the step
    net, learn_info = (None, None) if args.no_learned else \
        train_learned_guess(g, evecs, eps, two_m, cfg["seed_eig"])
    kept = []

    def step_core(with_guess, sloppy=SLOPPY):
        hisq.hisq_prepare_source(g, two_m, ee, eo, y)
        hisq.hisq_deflate(g, ev32, eps, two_m, y, x)
        if with_guess:
            kept[:] = hisq.hisq_nn_guess(net, two_m, y, x,
                                         flags=hisq.HISQ_NN_NORMALIZE | hisq.HISQ_NN_BF16,
                                         evecs=ev32, evals=eps)
        res = hisq.hisq_cg_solve(g, two_m, y, x, tol=tol, sloppy_prec=sloppy, reliable_delta=0.1,
                                 evecs=ev32, evals=eps, tol_restart=1e-3)
        hisq.hisq_reconstruct_odd(g, two_m, x, eo, po)
        return res

    def step():
        return step_core(False)

    def step_fp64(xo):
        hisq.hisq_prepare_source(g, two_m, ee, eo, y)
        hisq.hisq_deflate(g, evecs, eps, two_m, y, xo)
        res = hisq.hisq_cg_solve(g, two_m, y, xo, tol=tol)
        hisq.hisq_reconstruct_odd(g, two_m, xo, eo, po)
        return res

    classes = ("dslash", "dslash_aux", "dslash_aux2", "dslash_f32", "dslash_f32_aux",
               "dslash_f32_aux2", "dslash_q16", "dslash_q16_aux", "dslash_h16", "dslash_h16_aux",
               "blas", "gemm")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # every PROFILE_PERIOD-th launch of each kernel class is bracketed by HIP
    # events on its stream: the sample costs little inside the timed region
    hisq.hisq_profile_enable(True, PROFILE_PERIOD)
    for cls in classes:
        hisq.hisq_profile_read(cls)
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    hisq.hisq_profile_enable(False)
    prof = {cls: hisq.hisq_profile_read(cls) for cls in classes}
    print(f"[bench] {args.steps} steps in {t_steps:.3f} s", flush=True)
    last = results[-1]
    true_res = max(max(r.true_residual) for r in results)
    assert all(all(r.converged) for r in results), "a timed solve did not converge"

    # live roofline of the CG's 16-bit half stencil over the timed region
    n_plain, ms_plain = prof["dslash_h16"]
    n_aux, ms_aux = prof["dslash_h16_aux"]
    bytes_total = (n_plain * dslash_alg_bytes(g.vh, nrhs, 0, 4, 2, 16)
                   + n_aux * dslash_alg_bytes(g.vh, nrhs, 1, 4, 2, 16))
    launches = n_plain + n_aux
    avg_ms = (ms_plain + ms_aux) / max(launches, 1)
    # GB/s = (bytes per launch) / (ms per launch * 1e-3) / 1e9
    hbm_achieved = bytes_total / max(launches, 1) / avg_ms / 1e6 if launches else None
    # the same launches in operations: 13 per algorithmic byte, below the ridge
    # of the int16 dot-product rate (157.3 T ops/s / 8 TB/s = 19.7), so the
    # bound is HBM bandwidth
    flops_launch = STENCIL_FLOPS_PER_SITE_RHS * nrhs * g.vh
    achieved = flops_launch / avg_ms / 1e9 if launches else None
    traffic = read_traffic()

    # the same step in FP64 throughout, and the mixed solutions against it
    x64 = torch.empty_like(ee)
    step_fp64(x64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r64 = step_fp64(x64)
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    diff = ((x - x64).abs().pow(2).sum(dim=(1, 2)).sqrt()
            / x64.abs().pow(2).sum(dim=(1, 2)).sqrt()).max().item()
    fp64 = {"solves_per_s": nrhs * args.steps / t_fp64, "iterations_per_source": r64.iterations,
            "max_true_residual": max(r64.true_residual),
            "path": "FP64 eigenvectors, single deflation, FP64 CG"}
    print(f"[bench] FP64 deflated: {fp64['solves_per_s']:.1f} solves/s", flush=True)

    # plain FP64 even-odd CG, no deflation, one source at a time
    plain = None
    if not args.no_plain_cg:
        ys = [y[j:j + 1].clone() for j in range(nrhs)]
        xs = torch.zeros((1, 3, g.vh), dtype=torch.complex128, device="cuda")
        hisq.hisq_cg_solve(g, two_m, ys[0], xs, tol=tol)  # warm-up
        its = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(nrhs):
            xs.zero_()
            its.append(hisq.hisq_cg_solve(g, two_m, ys[j], xs, tol=tol).iterations[0])
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        plain = {"solves_per_s": nrhs / t_plain, "mean_iterations": float(np.mean(its)),
                 "seconds": t_plain}
        print(f"[bench] plain CG {nrhs} solves in {t_plain:.3f} s", flush=True)

    # the step with the learned guess between deflation and CG, and the
    # guess's held-out loss
    learned = None
    if net is not None:
        xd = torch.empty_like(y)
        hisq.hisq_prepare_source(g, two_m, ee, eo, y)
        hisq.hisq_deflate(g, evecs, eps, two_m, y, xd)
        Ax = torch.empty_like(y)
        hisq.hisq_mdagm(g, two_m, xd, Ax)
        held_out, _ = hisq.hisq_nn_loss_grad(net, y - Ax, x64 - xd, hisq.HISQ_NN_NORMALIZE)
        del xd, Ax
        step_core(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rl = step_core(True)
        torch.cuda.synchronize()
        t_with = time.perf_counter() - t0
        assert all(rl.converged), "a learned-guess solve did not converge"
        learned = dict(learn_info)
        learned.update({
            "held_out_loss": held_out, "kept": list(kept),
            "iterations_per_source_with": rl.iterations,
            "iterations_per_source_without": last.iterations,
            "solves_per_s_with": nrhs * args.steps / t_with,
            "solves_per_s_without": nrhs * args.steps / t_steps,
            "path": ("the timed step plus the network correction (BF16 weights) projected "
                     "off the deflation space, between the deflation and the CG"),
        })
        net.close()
        print(f"[bench] with the learned guess: {learned['solves_per_s_with']:.1f} solves/s,"
              f" mean iterations {np.mean(rl.iterations):.1f} (without: "
              f"{np.mean(last.iterations):.1f})", flush=True)

    # the timed step with the sloppy operator reading FP32 or BF16 links
    sloppy_links = {}
    for name, sp, skip in (("fp32_vectors_16bit_links", hisq.HISQ_Q16, False),
                           ("fp32_links", F32, False), ("bf16_links", hisq.HISQ_BF16, args.no_bf16)):
        if skip:
            continue
        step_core(False, sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rb = step_core(False, sp)
        torch.cuda.synchronize()
        t_var = time.perf_counter() - t0
        assert all(rb.converged), f"a {name} solve did not converge"
        sloppy_links[name] = {"solves_per_s": nrhs * args.steps / t_var,
                              "iterations_per_source": rb.iterations,
                              "reliable_updates_per_source": rb.reliable_updates,
                              "max_true_residual": max(rb.true_residual)}
        print(f"[bench] sloppy operator with {name}: {nrhs * args.steps / t_var:.1f} solves/s, "
              f"mean iterations {np.mean(rb.iterations):.1f}", flush=True)

    scan = None if args.no_dslash_scan else dslash_scan()
    if scan:
        print(f"[bench] dslash 32^3x64: {scan['f64']['GB_s']:.0f} GB/s (f64), "
              f"{scan['f32']['GB_s']:.0f} GB/s (f32), {scan['bf16']['GB_s']:.0f} GB/s (bf16)",
              flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        gpath = os.path.join(ROOT, "tests", "golden", "oracle_16x16x16x32.json")
        if os.path.exists(gpath):
            cpu = cpu_baseline(cfg, json.load(open(gpath)))
            print(f"[bench] oracle on host: {cpu['value']:.4f} solves/s", flush=True)

    value = nrhs * args.steps / t_steps
    out = {
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
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "deflated-cg-16^3x32", "lattice": "16x16x16x32", "eps": 0.5,
                   "two_m": two_m, "sources_per_step": nrhs, "n_ev": n_ev, "tol": tol,
                   "path": ("FP32 eigenvectors; batched mixed-precision CG (FP32 arithmetic; "
                            "16-bit fixed-point links, search direction and A p with a norm "
                            "per site; FP32 residual and correction; FP64 reductions and "
                            "reliable updates, delta_rd 0.1), re-deflation at delta_tr "
                            "1e-3")},
        "roofline": {"bound": "hbm",
                     "kernel": "k_dslash<float, h16c, q16c> (half stencil, 16-bit vectors "
                               "and links, int16 dot products, FP32 accumulation, 12 RHS)",
                     "achieved": hbm_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": hbm_achieved / HBM_PEAK_GBS if hbm_achieved else None,
                     "traffic": traffic, "launches_timed": launches, "timed_every": PROFILE_PERIOD,
                     "avg_launch_us": avg_ms * 1e3,
                     "alg_bytes_per_launch": bytes_total / max(launches, 1),
                     "ops_per_launch": flops_launch,
                     "arith_intensity_op_per_byte": flops_launch / (bytes_total / max(launches, 1))
                     if launches else None,
                     "alu_achieved_Tops": achieved,
                     "alu_peak_Tops": DOT2_VALU_PEAK_TOPS,
                     "alu_frac": achieved / DOT2_VALU_PEAK_TOPS if achieved else None,
                     "peak_note": ("algorithmic bytes per launch / average launch time (HIP "
                                   "events) against 8 TB/s; ops = the 1146 flops per site and "
                                   "RHS of the FP32 stencil, here as int16 dot products "
                                   "(157.3 T ops/s, ridge 19.7 op/B)")},
        "cpu_baseline": cpu,
        "iterations_per_source": last.iterations,
        "reliable_updates_per_source": last.reliable_updates,
        "redeflations_per_source": last.redeflations,
        "max_true_residual": true_res,
        "max_rel_diff_vs_fp64_solution": diff,
        "deflated_fp64_cg": fp64,
        "plain_fp64_cg": plain,
        "learned_guess": learned,
        "sloppy_links_variants": sloppy_links,
        "speedup_vs_plain_fp64_cg": value / plain["solves_per_s"] if plain else None,
        "eigensolve": {"seconds": t_eig, "matvecs": est.matvecs, "restarts": est.restarts,
                       "cheb_degree": est.cheb_degree, "max_residual": est.max_residual,
                       "lambda_1": float(lam[0]), "lambda_64": float(lam[-1])},
        "gauge_pack_seconds": t_pack,
        "dslash_32x32x32x64": scan,
        "kernel_sample": {k: {"launches_timed": v[0], "avg_us": v[1] / v[0] * 1e3 if v[0] else None}
                          for k, v in prof.items()},
    }
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
