"""GPU parity at the full size of the benchmarked workload (16^3 x 32, eps 0.5,
2m = 0.01, 12 Gaussian sources, 64 eigenpairs, tol 1e-10), in the launch
configuration bench.py times, against values the oracle computes here or
stored by tests/golden/make_workload_16x16x16x32_golden.py (oracle only)."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from oracle import hisq_oracle as O
from paper_2502_00152_amd import inputs as I
from tests.gpu_util import Problem, dev, from_parity, host, to_parity

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_16x16x16x32.json")))
SOLUTIONS = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                        "oracle_solutions_16x16x16x32.json")))


@pytest.fixture(scope="module")
def wl():
    import torch
    from paper_2502_00152_amd import hisq
    cfg = I.workload(1)
    pr = Problem.from_workload(1)
    pr.cfg = cfg
    pr.g = pr.gauge()
    pr.eta = np.stack([I.gaussian_source(cfg["dims"], sd) for sd in cfg["seed_src"]])
    full = dev(pr.eta)
    pr.ee = torch.empty((12, 3, pr.g.vh), dtype=torch.complex128, device="cuda")
    pr.eo = torch.empty_like(pr.ee)
    hisq.hisq_spinor_split(pr.g, full, pr.ee, pr.eo)
    pr.y = torch.empty_like(pr.ee)
    hisq.hisq_prepare_source(pr.g, cfg["two_m"], pr.ee, pr.eo, pr.y)
    print("[16x16x16x32] setup done", flush=True)
    yield pr
    pr.g.close()


@pytest.fixture(scope="module")
def eig(wl):
    import torch
    from paper_2502_00152_amd import hisq
    cfg = wl.cfg
    ev = torch.empty((64, 3, wl.g.vh), dtype=torch.complex128, device="cuda")
    st, lam, stats = hisq.hisq_eigensolve(wl.g, cfg["two_m"], 64, ev, tol=1e-10,
                                          seed=cfg["seed_eig"])
    print(f"[16x16x16x32] eigensolve {stats.seconds:.2f}s restarts={stats.restarts} "
          f"matvecs={stats.matvecs} deg={stats.cheb_degree} a={stats.cheb_a:.4g} "
          f"maxres={stats.max_residual:.3g}", flush=True)
    return ev, lam, stats


def test_dslash_sampled_sites(wl):
    """12-RHS half stencil (the CG's launch configuration) at 300 random sites."""
    import torch
    from paper_2502_00152_amd import hisq
    dims = wl.dims
    out = torch.empty_like(wl.ee)
    hisq.hisq_dslash_eo(wl.g, 0, wl.eo, out)
    got = host(out)
    rng = np.random.default_rng(5)
    lex_even = np.nonzero(O.even_mask(dims).ravel())[0]
    X, Y, Z, T = dims
    worst = 0.0
    for lex in rng.choice(lex_even, 300, replace=False):
        x, y, z, t = lex % X, (lex // X) % Y, (lex // (X * Y)) % Z, lex // (X * Y * Z)
        for r in (0, 5, 11):
            ref = O.dslash_site(wl.F, wl.L, np.ascontiguousarray(wl.eta[r]), (x, y, z, t))
            g = got[r, :, lex >> 1]
            worst = max(worst, np.abs(g - ref).max() / np.abs(ref).max())
    assert worst <= 1e-13


def test_eigenpairs_match_oracle(wl, eig):
    ev, lam, stats = eig
    ref = np.array(GOLDEN["eigenvalues"])
    lmax = stats.lambda_max
    assert np.abs(lam - ref).max() <= 1e-10 * lmax
    # relative to each eigenvalue: a residual r <= tol lambda_max moves a
    # Rayleigh quotient by at most r^2 / gap, far below 1e-10 lambda_i here
    print(f"[16x16x16x32] largest relative eigenvalue difference "
          f"{(np.abs(lam - ref) / ref).max():.3e}", flush=True)
    assert (np.abs(lam - ref) <= 1e-10 * ref).all()
    V = host(ev)
    G = V.reshape(64, -1).conj() @ V.reshape(64, -1).T
    assert np.abs(G - np.eye(64)).max() <= 1e-12
    two_m = wl.cfg["two_m"]
    res = []
    for i in range(0, 64, 7):
        v = from_parity(V[i:i + 1], wl.dims, 0)[0]
        res.append(O.norm(O.apply_A(wl.F, wl.L, two_m, v) - lam[i] * v))
    assert max(res) <= 1e-10 * lmax


def test_block_eigensolve_matches_oracle(wl, eig):
    """Block thick-restart Lanczos (12 vectors per step, the multi-RHS stencil
    launch of the CG) gives the same 64 pairs: eigenvalues against the
    oracle's ARPACK values, orthonormality and oracle residuals of sampled
    vectors, with fewer stencil launches than one vector per step."""
    import torch
    from paper_2502_00152_amd import hisq
    cfg = wl.cfg
    two_m = cfg["two_m"]
    ev = torch.empty((64, 3, wl.g.vh), dtype=torch.complex128, device="cuda")
    st, lam, stats = hisq.hisq_eigensolve(wl.g, two_m, 64, ev, tol=1e-10, seed=cfg["seed_eig"],
                                          block=12)
    print(f"[16x16x16x32] block 12 eigensolve {stats.seconds:.2f}s restarts={stats.restarts} "
          f"matvecs={stats.matvecs} (one vector per step: {eig[2].matvecs}) "
          f"maxres={stats.max_residual:.3g}", flush=True)
    ref = np.array(GOLDEN["eigenvalues"])
    lmax = stats.lambda_max
    assert np.abs(lam - ref).max() <= 1e-10 * lmax
    assert (np.abs(lam - ref) <= 1e-10 * ref).all()
    V = host(ev)
    G = V.reshape(64, -1).conj() @ V.reshape(64, -1).T
    assert np.abs(G - np.eye(64)).max() <= 1e-12
    res = []
    for i in range(3, 64, 9):
        v = from_parity(V[i:i + 1], wl.dims, 0)[0]
        res.append(O.norm(O.apply_A(wl.F, wl.L, two_m, v) - lam[i] * v))
    assert max(res) <= 1e-10 * lmax


def test_deflated_batched_cg(wl, eig):
    """The benchmarked step: deflate, batched CG on 12 sources, reconstruct."""
    import torch
    from paper_2502_00152_amd import hisq
    ev, lam, stats = eig
    cfg = wl.cfg
    two_m = cfg["two_m"]
    x = torch.empty_like(wl.y)
    hisq.hisq_deflate(wl.g, ev, lam - two_m ** 2, two_m, wl.y, x)
    res = hisq.hisq_cg_solve(wl.g, two_m, wl.y, x, tol=1e-10)
    assert all(res.converged)
    it0 = GOLDEN["cg_iterations_deflated"]
    assert abs(res.iterations[0] - it0) <= max(2, 0.01 * it0)
    xs, ys = host(x), host(wl.y)
    for r in range(12):
        xe = from_parity(xs[r:r + 1], wl.dims, 0)[0]
        ye = from_parity(ys[r:r + 1], wl.dims, 0)[0]
        tr = O.norm(ye - O.apply_A(wl.F, wl.L, two_m, xe)) / O.norm(ye)
        assert tr <= 1e-10, (r, tr)
    # full-lattice solution: M psi = eta up to (even residual)/(2m)
    po = torch.empty_like(wl.eo)
    hisq.hisq_reconstruct_odd(wl.g, two_m, x, wl.eo, po)
    psi = from_parity(xs[:1], wl.dims, 0)[0] + from_parity(host(po)[:1], wl.dims, 1)[0]
    r = O.apply_M(wl.F, wl.L, two_m, psi) - wl.eta[0]
    assert O.norm(r) <= 1e-10 * O.norm(ys[0]) / two_m * 1.01


def test_plain_cg_iterations(wl):
    import torch
    from paper_2502_00152_amd import hisq
    x = torch.zeros((1, 3, wl.g.vh), dtype=torch.complex128, device="cuda")
    res = hisq.hisq_cg_solve(wl.g, wl.cfg["two_m"], wl.y[:1].clone(), x, tol=1e-10)
    it0 = GOLDEN["cg_iterations_undeflated"]
    assert abs(res.iterations[0] - it0) <= max(2, 0.01 * it0)


def test_fp32_eigenvectors_stall_and_multi_deflation_recovers(wl, eig):
    """Section 3, Fig. 2 on the synthetic workload: with single-precision
    eigenvectors a single deflation leaves low-mode components at the FP32
    rounding level and the mixed-precision CG needs more iterations than with
    FP64 eigenvectors; re-deflating whenever the residual has fallen by
    delta_tr = 1e-3 recovers the FP64 iteration count.  Every solve meets the
    FP64 true residual 1e-10 (oracle-evaluated on two sources) and differs
    from the FP64 path's solution by at most the residual bound
    ||x - x'|| <= (||r|| + ||r'||) / lambda_1."""
    import torch
    from paper_2502_00152_amd import hisq
    ev, lam, stats = eig
    cfg = wl.cfg
    two_m = cfg["two_m"]
    eps = lam - two_m ** 2
    ev32 = torch.empty(ev.shape, dtype=torch.complex64, device="cuda")
    hisq.hisq_convert_vectors(ev, ev32)
    F32 = hisq.HISQ_FP32

    def solve(defl, **kw):
        x = torch.empty_like(wl.y)
        hisq.hisq_deflate(wl.g, defl, eps, two_m, wl.y, x)
        r = hisq.hisq_cg_solve(wl.g, two_m, wl.y, x, tol=1e-10, **kw)
        assert all(r.converged)
        return x, r

    x64, r64 = solve(ev)                                       # FP64 path
    _, r_e64 = solve(ev, sloppy_prec=F32)                      # FP64 eigenvectors
    _, r_e32 = solve(ev32, sloppy_prec=F32)                    # FP32, one deflation
    x_m, r_m = solve(ev32, sloppy_prec=F32, evecs=ev32, evals=eps, tol_restart=1e-3)
    it64, ite64, ite32, itm = (max(r.iterations) for r in (r64, r_e64, r_e32, r_m))
    print(f"[16x16x16x32] iterations: FP64 {it64}, mixed+FP64 evecs {ite64}, "
          f"mixed+FP32 evecs {ite32}, multi-deflation {itm} ({r_m.redeflations[0]} re-deflations)",
          flush=True)
    assert ite32 > ite64 + 10                  # the stall of single-precision eigenvectors
    assert itm <= it64 * 1.05 + 5              # multi-deflation recovers the FP64 count
    assert itm < ite32 - 30
    assert min(r_m.redeflations) >= 1
    xs, ys, x64s = host(x_m), host(wl.y), host(x64)
    for r in (0, 7):
        xe = from_parity(xs[r:r + 1], wl.dims, 0)[0]
        ye = from_parity(ys[r:r + 1], wl.dims, 0)[0]
        tr = O.norm(ye - O.apply_A(wl.F, wl.L, two_m, xe)) / O.norm(ye)
        assert tr <= 1e-10, (r, tr)
    lam1 = GOLDEN["eigenvalues"][0]
    for r in range(12):
        bound = (r_m.true_residual[r] + r64.true_residual[r]) * np.linalg.norm(ys[r]) / lam1
        assert np.linalg.norm(xs[r] - x64s[r]) <= bound * 1.01, r


def test_q16_stencil_sampled_sites(wl):
    """The timed sloppy operator: 12-RHS half stencil with FP32 vectors and
    16-bit fixed-point links, at 300 random sites, within the quantisation
    bound (step / sqrt(2)) T + 300 u32 S (see tests/test_gpu_lowp.py)."""
    import torch
    from paper_2502_00152_amd import hisq
    from tests.gpu_util import abs_stencil_site
    dims = wl.dims
    e32 = wl.eo.to(torch.complex64)
    out = torch.empty_like(e32)
    hisq.hisq_dslash_eo(wl.g, 0, e32, out, prec=hisq.HISQ_Q16)
    got = host(out).astype(np.complex128)
    eo32 = host(e32).astype(np.complex128)
    step = max(np.abs(wl.F.real).max(), np.abs(wl.F.imag).max(),
               np.abs(wl.L.real).max(), np.abs(wl.L.imag).max()) / 32767.0
    ones = np.ones((4,) + wl.F.shape[1:], dtype=np.complex128)
    rng = np.random.default_rng(6)
    lex_even = np.nonzero(O.even_mask(dims).ravel())[0]
    X, Y, Z, T = dims
    worst = 0.0
    for r in (0, 5, 11):
        psi = from_parity(eo32[r:r + 1], dims, 1)[0]
        for lex in rng.choice(lex_even, 100, replace=False):
            site = (lex % X, (lex // X) % Y, (lex // (X * Y)) % Z, lex // (X * Y * Z))
            ref = O.dslash_site(wl.F, wl.L, psi, site)
            S = abs_stencil_site(wl.F, wl.L, psi, site)
            Tq = abs_stencil_site(ones, ones, psi, site)
            err = np.abs(got[r, :, lex >> 1] - ref)
            bound = step / np.sqrt(2) * Tq + 300 * 2.0 ** -24 * S
            assert (err <= bound).all(), (r, site)
            worst = max(worst, float((err / bound).max()))
    print(f"[16x16x16x32] q16 stencil: worst error / bound {worst:.3f}", flush=True)


def test_half_stencil_sampled_sites(wl):
    """The timed sloppy stencil itself: 12 RHS rounded to 16-bit fixed point
    with one norm per site, 16-bit links (step = largest link component /
    qmax, see tests/gpu_util.py), integer products, output rounded to its site norm, at 300 random
    sites, within (step / sqrt 2) T + |D| w + 200 u32 S + m_o / 65534 (see
    tests/test_gpu_lowp.py)."""
    import torch
    from paper_2502_00152_amd import hisq
    from tests.gpu_util import abs_stencil_site, half_link_step
    dims = wl.dims
    e32 = wl.eo.to(torch.complex64)
    out = torch.empty_like(e32)
    hisq.hisq_dslash_eo(wl.g, 0, e32, out, prec=hisq.HISQ_HALF)
    got = host(out).astype(np.complex128)
    eo32 = host(e32).astype(np.complex128)
    step = half_link_step(wl.F, wl.L)
    ones = np.ones((4,) + wl.F.shape[1:], dtype=np.complex128)
    rng = np.random.default_rng(7)
    lex_even = np.nonzero(O.even_mask(dims).ravel())[0]
    X, Y, Z, T = dims
    worst = 0.0
    for r in (0, 5, 11):
        psi = from_parity(eo32[r:r + 1], dims, 1)[0]
        m = np.maximum(np.abs(psi.real), np.abs(psi.imag)).max(axis=-1, keepdims=True)
        w = np.sqrt(2) * m / 65534.0 * np.ones(psi.shape)
        for lex in rng.choice(lex_even, 100, replace=False):
            site = (lex % X, (lex // X) % Y, (lex // (X * Y)) % Z, lex // (X * Y * Z))
            ref = O.dslash_site(wl.F, wl.L, psi, site)
            S = abs_stencil_site(wl.F, wl.L, psi, site)
            Tq = abs_stencil_site(ones, ones, psi, site)
            Wq = abs_stencil_site(wl.F, wl.L, w, site)
            B = step / np.sqrt(2) * Tq + 1.01 * Wq + 200 * 2.0 ** -24 * S
            mo = 1.01 * (max(np.abs(ref.real).max(), np.abs(ref.imag).max()) + B.max()) / 65534.0
            err = np.abs(got[r, :, lex >> 1] - ref)
            bound = B + mo
            assert (err <= bound).all(), (r, site)
            worst = max(worst, float((err / bound).max()))
    print(f"[16x16x16x32] 16-bit stencil: worst error / bound {worst:.3f}", flush=True)
    assert worst > 0.05


@pytest.mark.parametrize("sloppy", ["q16", "half"])
def test_timed_step_16bit_multi_deflation(wl, eig, sloppy):
    """The timed step of the benchmark: FP32 eigenvectors, mixed CG whose
    sloppy operator reads 16-bit links (and, for "half", whose p and A p are
    held in 16 bits), re-deflation at delta_tr = 1e-3.
    Oracle-evaluated FP64 true residual <= 1e-10 on two sources, the solution
    within (||r|| + ||r'||) / lambda_1 of the FP64 path's, and the iteration
    count of the FP32-link path."""
    import torch
    from paper_2502_00152_amd import hisq
    ev, lam, stats = eig
    two_m = wl.cfg["two_m"]
    eps = lam - two_m ** 2
    ev32 = torch.empty(ev.shape, dtype=torch.complex64, device="cuda")
    hisq.hisq_convert_vectors(ev, ev32)

    def solve(defl, **kw):
        x = torch.empty_like(wl.y)
        hisq.hisq_deflate(wl.g, defl, eps, two_m, wl.y, x)
        r = hisq.hisq_cg_solve(wl.g, two_m, wl.y, x, tol=1e-10, **kw)
        assert all(r.converged)
        return x, r

    x64, r64 = solve(ev)
    kw = dict(reliable_delta=0.1, evecs=ev32, evals=eps, tol_restart=1e-3)
    sp = hisq.HISQ_Q16 if sloppy == "q16" else hisq.HISQ_HALF
    xq, rq = solve(ev32, sloppy_prec=sp, **kw)
    _, rf = solve(ev32, sloppy_prec=hisq.HISQ_FP32, **kw)
    print(f"[16x16x16x32] timed step iterations: {sloppy} {max(rq.iterations)}, "
          f"fp32 links {max(rf.iterations)}, fp64 {max(r64.iterations)}", flush=True)
    assert max(rq.iterations) <= max(rf.iterations) + 3
    xs, ys, x64s = host(xq), host(wl.y), host(x64)
    for r in (0, 11):
        xe = from_parity(xs[r:r + 1], wl.dims, 0)[0]
        ye = from_parity(ys[r:r + 1], wl.dims, 0)[0]
        tr = O.norm(ye - O.apply_A(wl.F, wl.L, two_m, xe)) / O.norm(ye)
        assert tr <= 1e-10, (r, tr)
    lam1 = GOLDEN["eigenvalues"][0]
    for r in range(12):
        bound = (rq.true_residual[r] + r64.true_residual[r]) * np.linalg.norm(ys[r]) / lam1
        assert np.linalg.norm(xs[r] - x64s[r]) <= bound * 1.01, r


def test_fp64_solution_matches_oracle_reference(wl, eig):
    """FP64 solution parity at the full size: sources 0 and 1, deflated FP64
    CG stopped at a true residual of 1e-13 (min(1e-10, 1e-9 / kappa) with
    kappa = lambda_max / lambda_1 ~ 7e3, floored at 1e-13), against the
    oracle's plain CG solution to 1e-14 stored by
    tests/golden/make_solutions_16x16x16x32_golden.py: the solution at 128
    seeded sites and its inner products with 8 seeded Gaussian vectors, each
    within 1e-9 relative."""
    import torch
    from paper_2502_00152_amd import hisq
    ev, lam, stats = eig
    two_m = wl.cfg["two_m"]
    sites = np.array(SOLUTIONS["sites_lex"])
    probes = np.stack([to_parity(np.where(O.even_mask(wl.dims)[..., None],
                                          I.gaussian_source(wl.dims, sd), 0), wl.dims, 0)[0]
                       for sd in SOLUTIONS["probe_seeds"]])
    y = wl.y[:2].clone()
    x = torch.empty_like(y)
    hisq.hisq_deflate(wl.g, ev, lam - two_m ** 2, two_m, y, x)
    res = hisq.hisq_cg_solve(wl.g, two_m, y, x, tol=1e-13)
    assert all(res.converged)
    xs = host(x)
    for k, ref in enumerate(SOLUTIONS["solutions"]):
        assert ref["source"] == k and ref["true_residual"] <= 1e-14
        got = xs[k][:, sites >> 1].T                        # [site][colour]
        want = np.array(ref["site_values_re"]) + 1j * np.array(ref["site_values_im"])
        e_sites = np.linalg.norm(got - want) / np.linalg.norm(want)
        pr_got = probes.reshape(len(probes), -1).conj() @ xs[k].reshape(-1)
        pr_want = np.array(ref["probe_re"]) + 1j * np.array(ref["probe_im"])
        scale = np.linalg.norm(probes.reshape(len(probes), -1), axis=1) * ref["norm"]
        e_probe = (np.abs(pr_got - pr_want) / scale).max()
        e_norm = abs(np.linalg.norm(xs[k]) - ref["norm"]) / ref["norm"]
        print(f"[16x16x16x32] source {k}: {res.iterations[k]} iterations, reported residual "
              f"{res.true_residual[k]:.2e}; relative error at sites {e_sites:.2e}, "
              f"probes {e_probe:.2e}, norm {e_norm:.2e}", flush=True)
        assert e_sites <= 1e-9 and e_probe <= 1e-9 and e_norm <= 1e-9
