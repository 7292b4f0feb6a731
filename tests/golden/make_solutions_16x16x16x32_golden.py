"""Write tests/golden/oracle_solutions_16x16x16x32.json: oracle-only reference
solutions of the 16^3 x 32 workload (eps 0.5, 2m = 0.01) for Gaussian sources
0 and 1, solved far below the benchmark's tolerance so that a GPU solution can
be checked to a relative error of 1e-9 (the FP64 solution bar).

Calls only the oracle and the seeded input generators.  For each source it
runs the oracle's plain CG on A psi_e = y_e (section 2: even-odd system with a
true-residual stop) to a true residual of 1e-14 and stores, instead of the
whole 6 MB field:
  * the solution at 128 seeded even sites (all three colours),
  * its inner products <w_j, psi_e> with 8 seeded Gaussian even-site vectors,
  * ||psi_e|| and the oracle's true residual.
An error of relative size e in psi_e shows in these up to about e.

Run:  python tests/golden/make_solutions_16x16x16x32_golden.py   (a few minutes on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import hisq_oracle as O  # noqa: E402
from paper_2502_00152_amd import inputs as I  # noqa: E402

N_SITES = 128
N_PROBES = 8
SITE_SEED = 16032
PROBE_SEED0 = 16100  # probe j uses gaussian_source(dims, PROBE_SEED0 + j), even sites kept
TOL = 1e-14


def sample_sites(dims):
    """Seeded even sites (lexicographic indices), sorted."""
    lex_even = np.nonzero(O.even_mask(dims).ravel())[0]
    rng = np.random.default_rng(SITE_SEED)
    return np.sort(rng.choice(lex_even, N_SITES, replace=False))


def probe(dims, j):
    w = I.gaussian_source(dims, PROBE_SEED0 + j)
    return np.where(O.even_mask(dims)[..., None], w, 0)


def main():
    cfg = I.workload(1)
    dims, two_m = cfg["dims"], cfg["two_m"]
    W = I.random_su3_field(dims, cfg["eps"], cfg["seed_fat"])
    N = I.random_su3_field(dims, cfg["eps"], cfg["seed_long"])
    F, L = O.fold_links(W, N, cfg["c_fat"], cfg["c_long"])
    sites = sample_sites(dims)
    probes = [probe(dims, j) for j in range(N_PROBES)]
    out = {
        "workload": "16x16x16x32 eps=0.5 2m=0.01, Gaussian sources 0 and 1",
        "generator": "tests/golden/make_solutions_16x16x16x32_golden.py "
                     "(oracle + seeded inputs only)",
        "two_m": two_m,
        "tol": TOL,
        "sites_lex": [int(s) for s in sites],
        "probe_seeds": [PROBE_SEED0 + j for j in range(N_PROBES)],
        "solutions": [],
        "oracle_threads": O.n_threads(),
    }
    for src in (0, 1):
        eta = I.gaussian_source(dims, cfg["seed_src"][src])
        y = O.source_even(F, L, two_m, eta)
        t0 = time.time()
        x, it, res = O.solve_even(F, L, two_m, y, tol=TOL, max_iter=5000)
        dt = time.time() - t0
        print(f"source {src}: {it} iterations, true residual {res:.3e}, {dt:.1f} s", flush=True)
        flat = x.reshape(-1, 3)
        vals = flat[sites]
        proj = [O.vdot(w, x) for w in probes]
        out["solutions"].append({
            "source": src,
            "iterations": int(it),
            "true_residual": float(res),
            "norm": O.norm(x),
            "y_norm": O.norm(y),
            "site_values_re": vals.real.tolist(),
            "site_values_im": vals.imag.tolist(),
            "probe_re": [p.real for p in proj],
            "probe_im": [p.imag for p in proj],
            "seconds": dt,
        })
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "oracle_solutions_16x16x16x32.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
