"""GPU parity of the odd-parity CG and of the full propagator solve (section 2:
even-odd preconditioning, reconstruction of the odd sites, and the CG polish
of the odd solution on (M^H M)_oo, as in the MILC + QUDA workflow; the
oracle's pins show that the full normal equation and Schur + reconstruction
agree).

Bars: oracle-evaluated residuals (the odd normal equation meets tol; the
library's reported ||eta - M psi|| / ||eta|| equals the oracle's to 1e-3), and
the solution error against the oracle's tight solve within the bound
||psi - psi*|| <= ||eta - M psi|| / (2m), since |eigenvalues of M| >= 2m
(D is anti-Hermitian).
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import hisq_oracle as O
from paper_2502_00152_amd import inputs as I
from tests.gpu_util import Problem, dev, from_parity, host, to_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def w8():
    cfg = I.workload(0)
    pr = Problem.from_workload(0)
    pr.g = pr.gauge()
    pr.two_m = cfg["two_m"]
    yield pr
    pr.g.close()


def point_sources(dims, sites):
    """3 colour point sources per site: the rows of a staggered propagator."""
    X, Y, Z, T = dims
    out = np.zeros((3 * len(sites), T, Z, Y, X, 3), dtype=np.complex128)
    for k, (x, y, z, t) in enumerate(sites):
        for c in range(3):
            out[3 * k + c, t, z, y, x, c] = 1.0
    return out


def A_odd(pr, v_full):
    """(2m)^2 v - D_oe D_eo v for an odd-site vector (zero on even sites)."""
    return pr.two_m ** 2 * v_full - O.d_oe(pr.F, pr.L, O.d_eo(pr.F, pr.L, v_full))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_odd_parity_cg(w8, prec):
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    b = to_parity(np.stack([I.gaussian_source(pr.dims, 77 + j) for j in range(2)]), pr.dims, 1)
    x = torch.zeros((2, 3, pr.g.vh), dtype=torch.complex128, device="cuda")
    sp = hisq.HISQ_FP64 if prec == "fp64" else hisq.HISQ_FP32
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, dev(b), x, tol=1e-10, parity=1, sloppy_prec=sp)
    assert all(res.converged)
    xs = host(x)
    for j in range(2):
        xf = from_parity(xs[j:j + 1], pr.dims, 1)[0]
        bf = from_parity(b[j:j + 1], pr.dims, 1)[0]
        tr = O.norm(bf - A_odd(pr, xf)) / O.norm(bf)
        assert tr <= 1e-10
        assert abs(tr - res.true_residual[j]) <= 1e-3 * tr
    with pytest.raises(hisq.HisqError):
        hisq.hisq_cg_solve(pr.g, pr.two_m, dev(b), x, parity=2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_propagator_two_point_sources_three_colours(w8, prec):
    """2 propagators x 3 colours (source points on an even and an odd site),
    without and with the odd polish."""
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    eta = point_sources(pr.dims, [(0, 0, 0, 0), (3, 2, 5, 1)])
    eta_d = dev(eta)
    sp = hisq.HISQ_FP64 if prec == "fp64" else hisq.HISQ_FP32
    exact = []
    for j in range(eta.shape[0]):
        ye = O.source_even(pr.F, pr.L, pr.two_m, eta[j])
        xe, _, _ = O.solve_even(pr.F, pr.L, pr.two_m, ye, tol=1e-14)
        exact.append(xe + O.reconstruct_odd(pr.F, pr.L, pr.two_m, xe, eta[j]))
    out = {}
    for polish in (0.0, 1e-10):
        psi = torch.empty_like(eta_d)
        r = hisq.hisq_propagator_solve(pr.g, pr.two_m, eta_d, psi, tol=1e-10, sloppy_prec=sp,
                                       polish_tol=polish)
        assert all(r.even.converged)
        if polish:
            assert all(r.polish.converged)
            assert max(r.polish.iterations) < max(r.even.iterations)
        ps = host(psi)
        for j in range(eta.shape[0]):
            res = O.norm(eta[j] - O.apply_M(pr.F, pr.L, pr.two_m, ps[j])) / O.norm(eta[j])
            assert abs(res - r.residual[j]) <= 1e-3 * res + 1e-15, (polish, j)
            err = O.norm(ps[j] - exact[j])
            assert err <= res * O.norm(eta[j]) / pr.two_m * 1.01 + 1e-12 * O.norm(exact[j])
        out[polish] = (r, [O.norm(ps[j] - exact[j]) / O.norm(exact[j]) for j in range(eta.shape[0])])
    # without the polish the odd rows hold exactly, the even rows carry ||r_e|| / (2m)
    r0, err0 = out[0.0]
    assert all(abs(a - b) <= 1e-12 + 1e-9 * a for a, b in zip(r0.residual, r0.residual_even))
    r1, err1 = out[1e-10]
    assert max(err1) <= max(err0) * 1.5 + 1e-12


def test_propagator_rejects_bad_arguments(w8):
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    eta = dev(point_sources(pr.dims, [(0, 0, 0, 0)]))
    with pytest.raises(hisq.HisqError):
        hisq.hisq_propagator_solve(pr.g, pr.two_m, eta, eta)
    with pytest.raises(hisq.HisqError):
        hisq.hisq_propagator_solve(pr.g, 0.0, eta, torch.empty_like(eta))
    with pytest.raises(hisq.HisqError):
        hisq.hisq_propagator_solve(pr.g, pr.two_m, eta, torch.empty_like(eta), polish_tol=-1.0)
