"""Write tests/golden/oracle_16x16x16x32.json: oracle-only reference values for the
16^3 x 32 deflated-CG workload (eps 0.5, 2m = 0.01, Gaussian source 0).

Calls only the oracle and the seeded input generators:
  * the 64 lowest eigenvalues of A = (2m)^2 - D_eo D_oe (ARPACK on the oracle's A),
    plus the 65th to report the gap at the cut;
  * the oracle CG iteration counts for source 0 to a true residual of 1e-10,
    undeflated and deflated with the oracle's own eigenvectors (Eq. (4)).
Run:  python tests/golden/make_workload_16x16x16x32_golden.py   (several minutes on 8 cores)
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


def main():
    cfg = I.workload(1)
    dims, two_m = cfg["dims"], cfg["two_m"]
    W = I.random_su3_field(dims, cfg["eps"], cfg["seed_fat"])
    N = I.random_su3_field(dims, cfg["eps"], cfg["seed_long"])
    F, L = O.fold_links(W, N, cfg["c_fat"], cfg["c_long"])
    eta = I.gaussian_source(dims, cfg["seed_src"][0])
    y = O.source_even(F, L, two_m, eta)

    t0 = time.time()
    _, it_plain, res_plain = O.solve_even(F, L, two_m, y, tol=cfg["tol"])
    t_plain = time.time() - t0
    print(f"undeflated CG: {it_plain} iterations, true residual {res_plain:.3e}, {t_plain:.1f} s",
          flush=True)

    k = cfg["n_ev"]
    n = 3 * int(np.prod(dims)) // 2
    t0 = time.time()
    w, V = O.lowest_eigenpairs(F, L, two_m, k + 1, method="arpack", tol=1e-12,
                               v0=np.ones(n, dtype=np.complex128))
    t_eig = time.time() - t0
    print(f"eigsh: {t_eig:.1f} s, lambda_1 = {w[0]:.6e}, lambda_{k} = {w[k - 1]:.6e}, "
          f"lambda_{k + 1} = {w[k]:.6e}", flush=True)
    x0 = O.from_compact(O.deflation_guess(V[:, :k], w[:k], O.to_compact(y, dims)), dims)
    t0 = time.time()
    _, it_defl, res_defl = O.solve_even(F, L, two_m, y, x0=x0, tol=cfg["tol"])
    t_defl = time.time() - t0
    print(f"deflated CG: {it_defl} iterations, true residual {res_defl:.3e}, {t_defl:.1f} s",
          flush=True)
    out = {
        "workload": "16x16x16x32 eps=0.5 2m=0.01, Gaussian source 0, tol 1e-10",
        "generator": "tests/golden/make_workload_16x16x16x32_golden.py (oracle + seeded inputs only)",
        "two_m": two_m,
        "eigenvalues": [float(v) for v in w[:k]],
        "eigenvalue_next": float(w[k]),
        "cg_iterations_undeflated": int(it_plain),
        "cg_iterations_deflated": int(it_defl),
        "true_residual_undeflated": float(res_plain),
        "true_residual_deflated": float(res_defl),
        "oracle_seconds": {"cg_undeflated": t_plain, "eigsh": t_eig, "cg_deflated": t_defl},
        "oracle_threads": O.n_threads(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_16x16x16x32.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
