"""GPU parity of the reduced-precision storage formats: BF16 (conversions,
the half stencil and M^H M with BF16 vectors and links, FP32 arithmetic),
16-bit fixed-point links (HISQ_Q16: FP32 vectors and arithmetic), the 16-bit
stencil of the HISQ_HALF CG (16-bit vectors and links, integer products), and
the mixed-precision CG whose sloppy operator reads BF16 or 16-bit links (sections
2-3: the bulk of the operator in reduced precision, FP64 restored at
reliable updates).

Q16 bar: each link component carries an absolute error <= step / 2 (step =
largest link component / 32767), i.e. <= step / sqrt(2) per complex entry,
so |out - D psi| <= (step / sqrt(2)) T + 300 u32 S with T = sum over the 16
hops and 3 colours of |psi| (the stencil with unit-modulus links) and the
FP32 arithmetic bound of the FP32 stencil; for M^H M both stencils and the
FP32 temporary enter, see the test.

Bars, derived from the arithmetic.  bfloat16 keeps 8 significant bits: round
to nearest gives a relative error u = 2^-8 per stored real.  The tests feed
the stencil inputs that are exactly representable in BF16 (rounded on the host
by torch), so the oracle sees the values the kernel reads.  Each of the 48
complex products of an output component uses one rounded link entry (error
<= u |U|), the FP32 accumulation adds at most gamma_96(FP32) < 6e-6 relative,
and the stored output is rounded once more (u |out|); hence
|out - D psi| <= (u + u + 6e-6 + u^2) (|D| |psi|) < 2.01 u S, S = |D| |psi|
componentwise.  For A = (2m)^2 - D_eo D_oe the odd temporary is stored in
BF16 too: |err| <= 2.01 u |D_eo| |D_oe| |v| (temporary) + 2.01 u |D_eo| |D_oe|
|v| (second stencil) + u (2m)^2 |v| + u |out| <= 5.1 u ((2m)^2 |v| + |D_eo|
|D_oe| |v|).  The conversions are checked bit for bit against an exact
round-to-nearest-even written out with frexp.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import hisq_oracle as O
from paper_2502_00152_amd import inputs as I
from tests.gpu_util import Problem, abs_stencil, dev, from_parity, half_link_step, host, to_parity

pytestmark = pytest.mark.gpu

UB = 2.0 ** -8
LATTICES = [((2, 2, 2, 2), 0.5), ((4, 6, 8, 10), 0.5), ((8, 8, 8, 8), 0.3)]


def bf16_rne(x):
    """Round float64 values to the nearest bfloat16 (8 significant bits, ties
    to even), exactly: x = m 2^e with 1/2 <= |m| < 1, keep 8 bits of m."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    sc = m * 256.0
    lo = np.floor(sc)
    fr = sc - lo
    r = np.where(fr > 0.5, lo + 1, np.where(fr < 0.5, lo, np.where(lo % 2 == 0, lo, lo + 1)))
    return np.ldexp(r / 256.0, e)


def to_bf16_tensor(v):
    """complex128 numpy [..] -> bfloat16 torch [.., 2] on the device (torch
    rounds on the host) and the exact values it holds, as complex128."""
    import torch
    pairs = np.stack([v.real, v.imag], axis=-1)
    t = torch.from_numpy(np.ascontiguousarray(pairs)).to(torch.bfloat16)
    exact = t.to(torch.float64).numpy()
    return t.cuda(), exact[..., 0] + 1j * exact[..., 1]


def from_bf16_tensor(t):
    import torch
    torch.cuda.synchronize()
    a = t.cpu().to(torch.float64).numpy()
    return a[..., 0] + 1j * a[..., 1]


def sources(dims, n, seed0):
    return np.stack([I.gaussian_source(dims, seed0 + j) for j in range(n)])


@pytest.fixture(scope="module", params=LATTICES, ids=lambda p: "x".join(map(str, p[0])))
def prob(request):
    dims, eps = request.param
    pr = Problem(dims, eps, 2101, 2102)
    pr.g = pr.gauge()
    yield pr
    pr.g.close()


def test_conversions_round_to_nearest_even():
    import torch
    from paper_2502_00152_amd import hisq
    rng = np.random.default_rng(5)
    vals = rng.standard_normal(4000) * np.exp(rng.uniform(-20, 20, 4000))
    # exact ties and values just off a tie, below FP32 resolution: a double
    # rounding through FP32 would get the latter wrong
    k = np.arange(128, 256, dtype=np.float64)
    ties = (k + 0.5) / 256.0 * 2.0 ** rng.integers(-30, 30, k.size)
    near = (k + 0.5 + 2.0 ** -40) / 256.0 * 2.0 ** rng.integers(-30, 30, k.size)
    allv = np.concatenate([vals, ties, -ties, near, -near])
    n = allv.size // 2 * 2
    z = (allv[:n:2] + 1j * allv[1:n:2]).reshape(1, -1)
    want = bf16_rne(z.real) + 1j * bf16_rne(z.imag)
    src = dev(z)
    dst = torch.empty((1, z.shape[1], 2), dtype=torch.bfloat16, device="cuda")
    hisq.hisq_convert_vectors(src, dst)
    got = from_bf16_tensor(dst)
    assert np.array_equal(got, want)
    # FP32 -> BF16 (the FP32 values are exact in float64: same rule)
    z32 = z.astype(np.complex64)
    hisq.hisq_convert_vectors(dev(z32), dst)
    assert np.array_equal(from_bf16_tensor(dst),
                          bf16_rne(z32.real.astype(np.float64)) + 1j * bf16_rne(z32.imag.astype(np.float64)))
    # BF16 -> FP64 and FP32 are exact
    back = torch.empty_like(src)
    hisq.hisq_convert_vectors(dst, back)
    assert np.array_equal(host(back), from_bf16_tensor(dst))
    back32 = torch.empty((1, z.shape[1]), dtype=torch.complex64, device="cuda")
    hisq.hisq_convert_vectors(dst, back32)
    assert np.array_equal(host(back32).astype(np.complex128), from_bf16_tensor(dst))


@pytest.mark.parametrize("nrhs", [1, 5, 12])
@pytest.mark.parametrize("out_parity", [0, 1])
def test_dslash_bf16_within_rounding_bound(prob, nrhs, out_parity):
    import torch
    from paper_2502_00152_amd import hisq
    dims = prob.dims
    in_par = 1 - out_parity
    inp, exact = to_bf16_tensor(to_parity(sources(dims, nrhs, 400), dims, in_par))
    out = torch.empty_like(inp)
    hisq.hisq_dslash_eo(prob.g, out_parity, inp, out)
    got = from_bf16_tensor(out)
    worst = 0.0
    for j in range(nrhs):
        full = from_parity(exact[j:j + 1], dims, in_par)[0]
        ref = to_parity(O.dslash(prob.F, prob.L, full, out_parity), dims, out_parity)[0]
        S = to_parity(abs_stencil(prob.F, prob.L, full), dims, out_parity)[0].real
        err = np.abs(got[j] - ref)
        assert (err <= 2.01 * UB * S + 1e-30).all(), (j, float((err / (S + 1e-300)).max() / UB))
        worst = max(worst, float((err / (S + 1e-300)).max()))
    # the links and the output really are BF16 (an FP32 path would be ~1e-6)
    assert worst > 0.05 * UB


@pytest.mark.parametrize("nrhs", [1, 4])
def test_mdagm_bf16_within_rounding_bound(prob, nrhs):
    import torch
    from paper_2502_00152_amd import hisq
    dims = prob.dims
    two_m = 0.07
    inp, exact = to_bf16_tensor(to_parity(sources(dims, nrhs, 420), dims, 0))
    out = torch.empty_like(inp)
    hisq.hisq_mdagm(prob.g, two_m, inp, out)
    got = from_bf16_tensor(out)
    for j in range(nrhs):
        full = from_parity(exact[j:j + 1], dims, 0)[0]
        ref = to_parity(O.apply_A(prob.F, prob.L, two_m, full), dims, 0)[0]
        odd = O.even_mask(dims)[..., None] == 0
        s1 = abs_stencil(prob.F, prob.L, full) * odd
        s2 = abs_stencil(prob.F, prob.L, s1)
        S = to_parity(s2 + two_m ** 2 * np.abs(full), dims, 0)[0].real
        err = np.abs(got[j] - ref)
        assert (err <= 5.1 * UB * S + 1e-30).all(), j


def test_bf16_stencil_shape_invariant():
    """Each output site sums its 16 hops in one order for every launch shape."""
    import torch
    from paper_2502_00152_amd import hisq
    dims = (4, 6, 8, 10)
    pr = Problem(dims, 0.5, 43, 44)
    g = pr.gauge()
    v, _ = to_bf16_tensor(to_parity(sources(dims, 12, 710), dims, 1))
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
    finally:
        hisq.hisq_set_tuning("dslash_rhs_per_thread", 0)
        hisq.hisq_set_tuning("dslash_lanes_per_site", 0)
        g.close()


# ----------------------------------------------- CG with a BF16-link operator
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


def test_cg_with_bf16_links_meets_fp64_residual(w8):
    """The convergence decision is taken on the FP64 true residual, so the
    reduced-precision operator changes the iteration count, not the answer:
    oracle-evaluated residual <= tol, and the solution within
    ||A^-1|| (r_gpu + r_oracle) ||b|| of the oracle's."""
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    tol = 1e-10
    bs = to_parity(pr.y, pr.dims, 0)
    b = dev(bs)
    x = torch.zeros_like(b)
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x, tol=tol, sloppy_prec=hisq.HISQ_BF16)
    assert all(res.converged)
    xs = host(x)
    x32 = torch.zeros_like(b)
    r32 = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x32, tol=tol, sloppy_prec=hisq.HISQ_FP32)
    for j in range(3):
        full = from_parity(xs[j:j + 1], pr.dims, 0)[0]
        tr = O.norm(pr.y[j] - O.apply_A(pr.F, pr.L, pr.two_m, full)) / O.norm(pr.y[j])
        assert tr <= tol
        xo, _, _ = O.solve_even(pr.F, pr.L, pr.two_m, pr.y[j], tol=1e-13)
        bound = (tr + 1e-13) * np.linalg.norm(bs[j]) / pr.two_m ** 2
        assert np.linalg.norm(xs[j] - to_parity(xo, pr.dims, 0)[0]) <= bound
    # more reliable updates than with FP32 links (each cycle gains less), and
    # a bounded iteration cost
    assert sum(res.reliable_updates) >= sum(r32.reliable_updates)
    assert max(res.iterations) <= 2 * max(r32.iterations) + 32


# ---------------------------------------------------- 16-bit fixed-point links
U32 = 2.0 ** -24


def q16_step(pr):
    return max(np.abs(pr.F.real).max(), np.abs(pr.F.imag).max(),
               np.abs(pr.L.real).max(), np.abs(pr.L.imag).max()) / 32767.0


@pytest.mark.parametrize("nrhs", [1, 5, 12])
@pytest.mark.parametrize("out_parity", [0, 1])
def test_dslash_q16_within_quantisation_bound(prob, nrhs, out_parity):
    import torch
    from paper_2502_00152_amd import hisq
    dims = prob.dims
    in_par = 1 - out_parity
    v32 = to_parity(sources(dims, nrhs, 440), dims, in_par).astype(np.complex64)
    inp = torch.from_numpy(v32).cuda()
    out = torch.empty_like(inp)
    hisq.hisq_dslash_eo(prob.g, out_parity, inp, out, prec=hisq.HISQ_Q16)
    got = host(out).astype(np.complex128)
    step = q16_step(prob)
    ones = np.ones_like(prob.F)
    worst = 0.0
    for j in range(nrhs):
        full = from_parity(v32[j:j + 1].astype(np.complex128), dims, in_par)[0]
        ref = to_parity(O.dslash(prob.F, prob.L, full, out_parity), dims, out_parity)[0]
        S = to_parity(abs_stencil(prob.F, prob.L, full), dims, out_parity)[0].real
        T = to_parity(abs_stencil(ones, ones, full), dims, out_parity)[0].real
        err = np.abs(got[j] - ref)
        bound = step / np.sqrt(2) * T + 300 * U32 * S
        assert (err <= bound + 1e-30).all(), (j, float((err / bound).max()))
        worst = max(worst, float((err / (step * T + 1e-300)).max()))
    assert worst > 0.01  # the links really are quantised (FP32 links: ~1e-3 of this)


@pytest.mark.parametrize("nrhs", [1, 4])
def test_mdagm_q16_within_quantisation_bound(prob, nrhs):
    import torch
    from paper_2502_00152_amd import hisq
    dims = prob.dims
    two_m = 0.07
    v32 = to_parity(sources(dims, nrhs, 460), dims, 0).astype(np.complex64)
    inp = torch.from_numpy(v32).cuda()
    out = torch.empty_like(inp)
    hisq.hisq_mdagm(prob.g, two_m, inp, out, prec=hisq.HISQ_Q16)
    got = host(out).astype(np.complex128)
    step = q16_step(prob)
    ones = np.ones_like(prob.F)
    odd = O.even_mask(dims)[..., None] == 0
    even = ~odd
    for j in range(nrhs):
        full = from_parity(v32[j:j + 1].astype(np.complex128), dims, 0)[0]
        ref = to_parity(O.apply_A(prob.F, prob.L, two_m, full), dims, 0)[0]
        s1 = abs_stencil(prob.F, prob.L, full) * odd                 # |D_oe| |v|
        t1 = abs_stencil(ones, ones, full) * odd                     # T_oe |v|
        S2 = abs_stencil(prob.F, prob.L, s1) + two_m ** 2 * np.abs(full)
        Tq = abs_stencil(prob.F, prob.L, t1) + abs_stencil(ones, ones, s1)
        bound = to_parity((step / np.sqrt(2) * Tq * 1.01 + 600 * U32 * S2) * even, dims, 0)[0].real
        err = np.abs(got[j] - ref)
        assert (err <= bound + 1e-30).all(), j


def test_cg_with_q16_links_keeps_fp32_iterations(w8):
    """With links accurate to ~4e-5 the sloppy recurrence loses almost nothing
    against FP32 links, and the answer is still decided by the FP64 true
    residual."""
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    tol = 1e-10
    bs = to_parity(pr.y, pr.dims, 0)
    b = dev(bs)
    x = torch.zeros_like(b)
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x, tol=tol, sloppy_prec=hisq.HISQ_Q16)
    assert all(res.converged)
    x32 = torch.zeros_like(b)
    r32 = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x32, tol=tol, sloppy_prec=hisq.HISQ_FP32)
    xs = host(x)
    for j in range(3):
        full = from_parity(xs[j:j + 1], pr.dims, 0)[0]
        tr = O.norm(pr.y[j] - O.apply_A(pr.F, pr.L, pr.two_m, full)) / O.norm(pr.y[j])
        assert tr <= tol
    assert max(res.iterations) <= 1.05 * max(r32.iterations) + 8, (res.iterations, r32.iterations)


# ------------------------------------- 16-bit vectors in the CG (HISQ_HALF)
def test_cg_with_half_vectors_meets_fp64_residual(w8):
    """p, A p and the odd temporary in 16-bit fixed point with one norm per
    site (~3e-5 relative), 16-bit links: the FP64 true residual decides, the
    iteration count stays that of FP32 vectors, and the solution is within
    ||A^-1|| (r_gpu + r_oracle) ||b|| of the oracle's."""
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    tol = 1e-10
    bs = to_parity(pr.y, pr.dims, 0)
    b = dev(bs)
    x = torch.zeros_like(b)
    res = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x, tol=tol, sloppy_prec=hisq.HISQ_HALF)
    assert all(res.converged)
    r32 = hisq.hisq_cg_solve(pr.g, pr.two_m, b, torch.zeros_like(b), tol=tol,
                             sloppy_prec=hisq.HISQ_FP32)
    xs = host(x)
    for j in range(3):
        full = from_parity(xs[j:j + 1], pr.dims, 0)[0]
        tr = O.norm(pr.y[j] - O.apply_A(pr.F, pr.L, pr.two_m, full)) / O.norm(pr.y[j])
        assert tr <= tol
        xo, _, _ = O.solve_even(pr.F, pr.L, pr.two_m, pr.y[j], tol=1e-13)
        bound = (tr + 1e-13) * np.linalg.norm(bs[j]) / pr.two_m ** 2
        assert np.linalg.norm(xs[j] - to_parity(xo, pr.dims, 0)[0]) <= bound
    assert max(res.iterations) <= 1.05 * max(r32.iterations) + 8, (res.iterations, r32.iterations)


def test_cg_half_batch_equals_single_solves(w8):
    """Quantisation is per (RHS, site) and the <p, Ap> partials are summed in
    one order for any launch shape, so a batch equals separate solves bitwise."""
    import torch
    from paper_2502_00152_amd import hisq
    pr = w8
    b = dev(to_parity(pr.y, pr.dims, 0))
    x = torch.zeros_like(b)
    rb = hisq.hisq_cg_solve(pr.g, pr.two_m, b, x, tol=1e-10, sloppy_prec=hisq.HISQ_HALF)
    for j in range(3):
        xj = torch.zeros_like(b[j:j + 1])
        rj = hisq.hisq_cg_solve(pr.g, pr.two_m, b[j:j + 1].clone(), xj, tol=1e-10,
                                sloppy_prec=hisq.HISQ_HALF)
        assert rj.iterations[0] == rb.iterations[j]
        assert torch.equal(xj[0], x[j])


# ------------------------------------- the 16-bit stencil itself (HISQ_HALF)
# The operators at HISQ_HALF take FP32 vectors, round them to 16-bit fixed
# point with one norm per site (|v - v'| <= m_y / 65534 per real component, m_y
# = the site's largest |component|), apply the CG's 16-bit stencil (links with
# step_n = largest folded link component / qmax, qmax chosen per field so that
# the integer dot products cannot overflow (see tests/gpu_util.py; ~26700 for
# these near-unitary links), |dU| <= step_n / 2 per real;
# integer products exact; FP32 accumulation) and store the result rounded to
# its own site norm (<= m_o / 65534 per real).  Componentwise, per output
# colour: |out - D v| <= (step_n / sqrt 2) T + |D| w + 200 u32 S + m_o / 65534,
# with T the stencil of |v| through unit links, w = sqrt 2 m_y / 65534 the
# per-site bound of |v - v'|, S = |D| |v|.
def qn_step(pr):
    return half_link_step(pr.F, pr.L)


def site_max(v):
    """Largest |Re| or |Im| over the three colours of each site, [..., 1]."""
    return np.maximum(np.abs(v.real), np.abs(v.imag)).max(axis=-1, keepdims=True)


def half_bound(pr, full, mo_extra=None):
    ones = np.ones_like(pr.F)
    T = abs_stencil(ones, ones, full)
    w = np.sqrt(2) * site_max(full) / 65534.0 * np.ones_like(np.abs(full))
    S = abs_stencil(pr.F, pr.L, full)
    return qn_step(pr) / np.sqrt(2) * T + 1.01 * abs_stencil(pr.F, pr.L, w) + 200 * U32 * S


@pytest.mark.parametrize("nrhs", [1, 5, 12])
@pytest.mark.parametrize("out_parity", [0, 1])
def test_dslash_half_within_quantisation_bound(prob, nrhs, out_parity):
    import torch
    from paper_2502_00152_amd import hisq
    dims = prob.dims
    in_par = 1 - out_parity
    v32 = to_parity(sources(dims, nrhs, 480), dims, in_par).astype(np.complex64)
    inp = torch.from_numpy(v32).cuda()
    out = torch.empty_like(inp)
    hisq.hisq_dslash_eo(prob.g, out_parity, inp, out, prec=hisq.HISQ_HALF)
    got = host(out).astype(np.complex128)
    worst = 0.0
    for j in range(nrhs):
        full = from_parity(v32[j:j + 1].astype(np.complex128), dims, in_par)[0]
        ref_full = O.dslash(prob.F, prob.L, full, out_parity)
        ref = to_parity(ref_full, dims, out_parity)[0]
        B = half_bound(prob, full)
        # the kernel's site norm is that of its own result, within B of ref
        mo = 1.01 * (site_max(ref_full) + B.max(axis=-1, keepdims=True)) / 65534.0
        bound = to_parity(B + mo, dims, out_parity)[0].real
        err = np.abs(got[j] - ref)
        assert (err <= bound + 1e-30).all(), (j, float((err / bound).max()))
        worst = max(worst, float((err / bound).max()))
    assert worst > 0.05  # the rounding is really there (an FP32 stencil: ~1e-3 of this)


@pytest.mark.parametrize("nrhs", [1, 4])
def test_mdagm_half_within_quantisation_bound(prob, nrhs):
    """A = (2m)^2 - D_eo D_oe with the odd temporary stored in 16 bits too: the
    first stencil's bound enters the second through |D_eo|, with the second's
    own link, arithmetic and output-rounding terms and (2m)^2 |v - v'|."""
    import torch
    from paper_2502_00152_amd import hisq
    dims = prob.dims
    two_m = 0.07
    v32 = to_parity(sources(dims, nrhs, 500), dims, 0).astype(np.complex64)
    inp = torch.from_numpy(v32).cuda()
    out = torch.empty_like(inp)
    hisq.hisq_mdagm(prob.g, two_m, inp, out, prec=hisq.HISQ_HALF)
    got = host(out).astype(np.complex128)
    odd = (O.even_mask(dims)[..., None] == 0)
    even = ~odd
    for j in range(nrhs):
        full = from_parity(v32[j:j + 1].astype(np.complex128), dims, 0)[0]
        t = O.dslash(prob.F, prob.L, full, 1) * odd
        B1 = half_bound(prob, full)
        Bt = (B1 + 1.01 * (site_max(t) + B1.max(axis=-1, keepdims=True)) / 65534.0) * odd
        ref_full = O.apply_A(prob.F, prob.L, two_m, full)
        ref = to_parity(ref_full, dims, 0)[0]
        # second stencil on t'' (|t''| <= |t| + Bt), (2m)^2 v' from the
        # rounded input, FP32 epilogue, output rounding
        ones = np.ones_like(prob.F)
        B2 = half_bound(prob, t) + 1.01 * abs_stencil(prob.F, prob.L, Bt)
        B2 = B2 + qn_step(prob) / np.sqrt(2) * abs_stencil(ones, ones, Bt)
        B2 = B2 + two_m ** 2 * (1.01 * np.sqrt(2) * site_max(full) / 65534.0 + 200 * U32 * np.abs(full))
        B2 = B2 + 1.01 * (site_max(ref_full) + B2.max(axis=-1, keepdims=True)) / 65534.0
        bound = to_parity(B2 * even, dims, 0)[0].real
        err = np.abs(got[j] - ref)
        assert (err <= bound + 1e-30).all(), (j, float((err / bound).max()))


def test_dslash_half_independent_of_launch_shape():
    """Exact integer products and one FP32 accumulation order per site: every
    launch shape gives the same bits."""
    import torch
    from paper_2502_00152_amd import hisq
    dims = (8, 8, 8, 12)
    pr = Problem(dims, 0.5, 2111, 2112)
    g = pr.gauge()
    v = torch.from_numpy(to_parity(sources(dims, 12, 520), dims, 1).astype(np.complex64)).cuda()
    ref = torch.empty_like(v)
    hisq.hisq_dslash_eo(g, 0, v, ref, prec=hisq.HISQ_HALF)
    shapes = [(nr, 1) for nr in (1, 2, 3, 4, 6, 12)] + [(nr, l) for l in (2, 4) for nr in (1, 3, 6)]
    try:
        for nr, lps in shapes:
            hisq.hisq_set_tuning("dslash_rhs_per_thread", nr)
            hisq.hisq_set_tuning("dslash_lanes_per_site", lps)
            out = torch.empty_like(v)
            hisq.hisq_dslash_eo(g, 0, v, out, prec=hisq.HISQ_HALF)
            assert torch.equal(out, ref), (nr, lps)
    finally:
        hisq.hisq_set_tuning("dslash_rhs_per_thread", 0)
        hisq.hisq_set_tuning("dslash_lanes_per_site", 0)
        g.close()


def test_dslash_half_integer_sums_at_their_bound(prob):
    """The worst case of the integer dot products: the input at the neighbour
    of the link row with the largest sum of |Re| + |Im| has every component at
    +-1 (the site's norm, stored as +-32767) with the signs of that row, so the
    real part of the row times it is the largest integer sum any vector can
    give.  An int32 overflow would put that output off by ~2^32 steps; it must
    stay within the quantisation bound."""
    import torch
    from paper_2502_00152_amd import hisq
    dims = prob.dims
    X, Y, Z, T = dims
    a = np.abs(prob.F.real) + np.abs(prob.F.imag)
    rowl1 = (a[..., 0] + a[..., 1]) + a[..., 2]           # [4][T][Z][Y][X][3]
    mu, t, z, y, x, row = np.unravel_index(int(np.argmax(rowl1)), rowl1.shape)
    site = [x, y, z, t]
    nb = list(site)
    nb[mu] = (nb[mu] + 1) % dims[mu]
    U = prob.F[mu, t, z, y, x, row]                        # the row, 3 complex
    psi = np.zeros((T, Z, Y, X, 3), dtype=np.complex128)
    psi[nb[3], nb[2], nb[1], nb[0]] = np.sign(U.real) - 1j * np.sign(U.imag)
    out_parity = int((x + y + z + t) % 2)
    in_par = 1 - out_parity
    v32 = to_parity(psi[None], dims, in_par).astype(np.complex64)
    inp = torch.from_numpy(v32).cuda()
    out = torch.empty_like(inp)
    hisq.hisq_dslash_eo(prob.g, out_parity, inp, out, prec=hisq.HISQ_HALF)
    got = host(out).astype(np.complex128)[0]
    ref_full = O.dslash(prob.F, prob.L, psi, out_parity)
    ref = to_parity(ref_full[None], dims, out_parity)[0]
    B = half_bound(prob, psi)
    mo = 1.01 * (site_max(ref_full) + B.max(axis=-1, keepdims=True)) / 65534.0
    bound = to_parity((B + mo)[None], dims, out_parity)[0].real
    err = np.abs(got - ref)
    assert (err <= bound + 1e-30).all(), float((err / bound).max())
    # the chosen output really is the extreme sum (real part = row L1 norm),
    # where no other hop of the site reaches the same neighbour
    if dims[mu] in (2, 4):
        return
    lex = ((t * Z + z) * Y + y) * X + x
    assert abs(ref[row, lex >> 1].real - rowl1[mu, t, z, y, x, row]) < 1e-12
    assert abs(got[row, lex >> 1].real - ref[row, lex >> 1].real) <= bound[row, lex >> 1]
