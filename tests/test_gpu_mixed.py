"""GPU parity of the FP32 (sloppy) operators and the mixed-precision CG
(section 2: the conventional solve is mixed-precision CG; section 3: reliable
updates with delta_rd = 0.1).

FP32 stencil bar, derived from the arithmetic: every output component is a
sum of 16 hops x 3 colours = 48 complex products, i.e. 96 real products per
real part; with FP32 links (rounded from FP64: relative error u = 2^-24 per
entry) and FMA accumulation, |error| <= 2 sqrt(2) (gamma_96 + u) S with
S = (|D| |psi|) componentwise, i.e. about 275 u S.  The tests use 280 u S for
one stencil and 600 u (|D_eo| |D_oe| |v| + (2m)^2 |v|) for A = (2m)^2 - D_eo D_oe.

Mixed CG bar: the oracle-evaluated FP64 true residual meets tol, and the
solution differs from the oracle's by at most ||A^-1|| (r_gpu + r_oracle)
<= (r_gpu + r_oracle) / (2m)^2 (the smallest eigenvalue of A is >= (2m)^2).
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import hisq_oracle as O
from paper_2502_00152_amd import inputs as I
from tests.gpu_util import Problem, abs_stencil, dev, from_parity, host, to_parity

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
LATTICES = [((2, 2, 2, 2), 0.5), ((4, 6, 8, 10), 0.5), ((8, 8, 8, 8), 0.3)]


def sources(dims, n, seed0):
    return np.stack([I.gaussian_source(dims, seed0 + j) for j in range(n)])


@pytest.fixture(scope="module", params=LATTICES, ids=lambda p: "x".join(map(str, p[0])))
def prob(request):
    dims, eps = request.param
    pr = Problem(dims, eps, 2001, 2002)
    pr.g = pr.gauge()
    yield pr
    pr.g.close()


@pytest.mark.parametrize("nrhs", [1, 5, 12])
@pytest.mark.parametrize("out_parity", [0, 1])
def test_dslash_fp32_within_rounding_bound(prob, nrhs, out_parity):
    import torch
    from paper_2502_00152_amd import hisq
    dims = prob.dims
    in_par = 1 - out_parity
    v32 = to_parity(sources(dims, nrhs, 300), dims, in_par).astype(np.complex64)
    inp = torch.from_numpy(v32).cuda()
    out = torch.empty_like(inp)
    hisq.hisq_dslash_eo(prob.g, out_parity, inp, out)
    got = host(out).astype(np.complex128)
    for j in range(nrhs):
        full = from_parity(v32[j:j + 1].astype(np.complex128), dims, in_par)[0]
        ref = to_parity(O.dslash(prob.F, prob.L, full, out_parity), dims, out_parity)[0]
        S = to_parity(abs_stencil(prob.F, prob.L, full), dims, out_parity)[0].real
        err = np.abs(got[j] - ref)
        assert (err <= 280 * U32 * S + 1e-30).all(), (j, float((err / (S + 1e-300)).max() / U32))


@pytest.mark.parametrize("nrhs", [1, 4])
def test_mdagm_fp32_within_rounding_bound(prob, nrhs):
    import torch
    from paper_2502_00152_amd import hisq
    dims = prob.dims
    two_m = 0.07
    v32 = to_parity(sources(dims, nrhs, 320), dims, 0).astype(np.complex64)
    inp = torch.from_numpy(v32).cuda()
    out = torch.empty_like(inp)
    hisq.hisq_mdagm(prob.g, two_m, inp, out)
    got = host(out).astype(np.complex128)
    for j in range(nrhs):
        full = from_parity(v32[j:j + 1].astype(np.complex128), dims, 0)[0]
        ref = to_parity(O.apply_A(prob.F, prob.L, two_m, full), dims, 0)[0]
        odd = O.even_mask(dims)[..., None] == 0
        s1 = abs_stencil(prob.F, prob.L, full) * odd          # |D_oe| |v| on odd sites
        s2 = abs_stencil(prob.F, prob.L, s1)                   # |D_eo| |D_oe| |v|
        S = to_parity(s2 + two_m ** 2 * np.abs(full), dims, 0)[0].real
        err = np.abs(got[j] - ref)
        assert (err <= 600 * U32 * S + 1e-30).all(), j


def test_fp32_stencil_grouping_is_bitwise_invariant():
    """The RHS grouping of the FP32 stencil changes only the launch shape."""
    import torch
    from paper_2502_00152_amd import hisq
    dims = (4, 6, 8, 10)
    pr = Problem(dims, 0.5, 43, 44)
    g = pr.gauge()
    v = torch.from_numpy(to_parity(sources(dims, 12, 700), dims, 1).astype(np.complex64)).cuda()
    ref = torch.empty_like(v)
    hisq.hisq_dslash_eo(g, 0, v, ref)
    shapes = [(nr, 1) for nr in (1, 2, 3, 4, 6, 12)] + [(nr, l) for l in (2, 4) for nr in (1, 3, 6)]
    try:
        for nr, lps in shapes:
            hisq.hisq_set_tuning("dslash_rhs_per_thread", nr)
            hisq.hisq_set_tuning("dslash_lanes_per_site", lps)
            out = torch.empty_like(v)
            hisq.hisq_dslash_eo(g, 0, v, out)
            assert torch.equal(out, ref), (nr, lps)
        one = torch.empty_like(v[:1])
        hisq.hisq_set_tuning("dslash_rhs_per_thread", 0)
        hisq.hisq_set_tuning("dslash_lanes_per_site", 0)
        hisq.hisq_dslash_eo(g, 0, v[5:6].clone(), one)
        assert torch.equal(one[0], ref[5])
    finally:
        hisq.hisq_set_tuning("dslash_rhs_per_thread", 0)
        hisq.hisq_set_tuning("dslash_lanes_per_site", 0)
        g.close()


# ------------------------------------------------------------- mixed CG
@pytest.fixture(scope="module")
def w8():
    cfg = I.workload(0)
    pr = Problem.from_workload(0)
    pr.g = pr.gauge()
    pr.two_m = cfg["two_m"]
    eta = np.stack([I.gaussian_source(cfg["dims"], cfg["seed_src"][0] + j) for j in range(3)])
    pr.y = np.stack([O.source_even(pr.F, pr.L, pr.two_m, e) for e in eta])
    yield pr
    pr.g.close()


def oracle_residual(pr, x_soa, b_soa):
    out = []
    for j in range(b_soa.shape[0]):
        x = from_parity(x_soa[j:j + 1], pr.dims, 0)[0]
        b = from_parity(b_soa[j:j + 1], pr.dims, 0)[0]
        out.append(O.norm(b - O.apply_A(pr.F, pr.L, pr.two_m, x)) / O.norm(b))
    return out


def test_mixed_cg_solution_matches_oracle(w8):
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    tol = 1e-10
    bs = to_parity(pr.y[0], pr.dims, 0)
    b = dev(bs)
    x = torch.zeros_like(b)
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x, tol=tol, sloppy_prec=hisq.HISQ_FP32)
    assert res.converged == [True]
    assert res.reliable_updates[0] >= 5  # delta_rd = 0.1 over 10 decades
    assert res.redeflations == [0]
    tr = oracle_residual(pr, host(x), bs)[0]
    assert tr <= tol
    assert abs(res.true_residual[0] - tr) <= 1e-3 * tr + 1e-16
    xo, it64, _ = O.solve_even(pr.F, pr.L, pr.two_m, pr.y[0], tol=1e-13)
    ref = to_parity(xo, pr.dims, 0)[0]
    bound = (tr + 1e-13) * np.linalg.norm(bs) / pr.two_m ** 2
    assert np.linalg.norm(host(x)[0] - ref) <= bound
    # FP32 iterations cost at most a modest increase over the FP64 recurrence
    _, it_fp64, _ = O.solve_even(pr.F, pr.L, pr.two_m, pr.y[0], tol=tol)
    assert res.iterations[0] <= 1.25 * it_fp64 + 16, (res.iterations[0], it_fp64)


def test_mixed_cg_batched_equals_single(w8):
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    bs = to_parity(pr.y, pr.dims, 0)
    b = dev(bs)
    x = torch.zeros_like(b)
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x, tol=1e-10, sloppy_prec=hisq.HISQ_FP32)
    assert all(res.converged)
    for j in range(3):
        xj = torch.zeros_like(b[j:j + 1])
        rj = hisq.hisq_cg_solve(pr.g, pr.two_m, b[j:j + 1].clone(), xj, tol=1e-10,
                                sloppy_prec=hisq.HISQ_FP32)
        assert rj.iterations[0] == res.iterations[j]
        assert rj.reliable_updates[0] == res.reliable_updates[j]
        assert torch.equal(xj[0], x[j])


def test_mixed_cg_reliable_interval_and_initial_guess(w8):
    """A periodic reliable update and a nonzero initial guess still reach tol."""
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    bs = to_parity(pr.y[1], pr.dims, 0)
    b = dev(bs)
    x0 = to_parity(0.3 * pr.y[2], pr.dims, 0)
    x = dev(x0)
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x, tol=1e-9, sloppy_prec=hisq.HISQ_FP32,
                             reliable_interval=20)
    assert res.converged == [True]
    assert res.reliable_updates[0] >= res.iterations[0] // 20
    assert oracle_residual(pr, host(x), bs)[0] <= 1e-9


def test_mixed_cg_edge_cases(w8):
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    F32 = hisq.HISQ_FP32
    bs = to_parity(pr.y[:2], pr.dims, 0)
    b = dev(bs)
    b[1].zero_()
    x = torch.ones_like(b)
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x, tol=1e-10, sloppy_prec=F32)
    assert res.converged == [True, True]
    assert torch.count_nonzero(x[1]) == 0          # b = 0 gives x = 0
    # max_iter reached: NOT_CONVERGED, residual reported
    x = torch.zeros_like(b[:1])
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, b[:1].clone(), x, tol=1e-10, max_iter=30,
                             sloppy_prec=F32, raise_on_fail=False)
    assert res.status == hisq.HISQ_ERR_NOT_CONVERGED
    assert res.iterations[0] <= 30 + 16 and not res.converged[0]
    tr = oracle_residual(pr, host(x), bs[:1])[0]
    assert abs(res.true_residual[0] - tr) <= 1e-6 * tr
    # max_iter = 0 leaves x at its initial value
    x = torch.zeros_like(b[:1])
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, b[:1].clone(), x, tol=1e-10, max_iter=0,
                             sloppy_prec=F32, raise_on_fail=False)
    assert res.status == hisq.HISQ_ERR_NOT_CONVERGED and torch.count_nonzero(x) == 0
    # invalid parameters
    for kw in ({"reliable_delta": 1.5}, {"reliable_interval": -1}, {"tol_restart": 1e-3},
               {"tol_restart": 2.0}):
        with pytest.raises(hisq.HisqError) as e:
            hisq.hisq_cg_solve(pr.g, pr.two_m, b[:1].clone(), torch.zeros_like(b[:1]),
                               sloppy_prec=F32, **kw)
        assert e.value.status == hisq.HISQ_ERR_INVALID_ARG, kw
    with pytest.raises(hisq.HisqError) as e:
        hisq.hisq_cg_solve(pr.g, pr.two_m, b[:1].clone(), torch.zeros_like(b[:1]),
                           sloppy_prec=99)
    assert e.value.status == hisq.HISQ_ERR_INVALID_ARG
    ev = torch.zeros((1, 3, pr.g.vh), dtype=torch.complex128, device="cuda")
    ev[0, 0, 0] = 1.0
    with pytest.raises(hisq.HisqError) as e:  # re-deflation needs the FP32 solver
        hisq.hisq_cg_solve(pr.g, pr.two_m, b[:1].clone(), torch.zeros_like(b[:1]),
                           evecs=ev, evals=[0.5], tol_restart=1e-3)
    assert e.value.status == hisq.HISQ_ERR_INVALID_ARG


def test_convert_vectors_rounds_to_nearest():
    """FP64 -> FP32 rounds each real to nearest (as numpy's cast does),
    FP32 -> FP64 is exact; bad arguments are rejected."""
    import torch
    from paper_2502_00152_amd import hisq
    rng = np.random.default_rng(3)
    v = (rng.standard_normal((5, 3, 1001)) + 1j * rng.standard_normal((5, 3, 1001))) * \
        np.exp(rng.uniform(-30, 30, (5, 3, 1001)))
    a = torch.from_numpy(v).cuda()
    b = torch.empty(a.shape, dtype=torch.complex64, device="cuda")
    hisq.hisq_convert_vectors(a, b)
    assert np.array_equal(host(b), v.astype(np.complex64))
    c = torch.empty_like(a)
    hisq.hisq_convert_vectors(b, c)
    assert np.array_equal(host(c), v.astype(np.complex64).astype(np.complex128))
    with pytest.raises(hisq.HisqError):
        hisq.hisq_convert_vectors(a, a)
    assert hisq.lib().hisq_convert_vectors(None, 0, None, 1, 4, None) == hisq.HISQ_ERR_INVALID_ARG
