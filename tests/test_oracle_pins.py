"""Pins of the oracle to facts the paper and the mathematics fix.

Each test states what it pins; a plausible mistake in the oracle (a dropped
term, a wrong sign or index, a transposed link) fails at least one of them.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import hisq_oracle as O
from paper_2502_00152_amd import inputs as I
from tests import pins

C1, C3 = I.C_FAT, I.C_LONG


def random_links(dims, eps=0.5, seed=11):
    W = I.random_su3_field(dims, eps, seed)
    N = I.random_su3_field(dims, eps, seed + 1)
    return O.fold_links(W, N, C1, C3)


def free_links(dims, c1=C1, c3=C3):
    U = I.unit_links(dims)
    return O.fold_links(U, U, c1, c3)


def rand_field(dims, seed):
    return I.gaussian_source(dims, seed)


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


# ---------------------------------------------------------------- stencil D
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 6, 8, 10), (6, 4, 4, 6)])
def test_anti_hermitian(dims):
    """<x, D y> = -<D x, y> for any links (D anti-Hermitian, section 2)."""
    F, L = random_links(dims)
    x, y = rand_field(dims, 1), rand_field(dims, 2)
    lhs = O.vdot(x, O.dslash(F, L, y))
    rhs = -O.vdot(O.dslash(F, L, x), y)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_anti_hermitian_parity_blocks():
    """<x_e, D_eo y_o> = -<D_oe x_e, y_o>, and the diagonal parity blocks vanish."""
    dims = (4, 6, 8, 10)
    F, L = random_links(dims)
    m = O.even_mask(dims)[..., None]
    xe = np.where(m, rand_field(dims, 3), 0)
    yo = np.where(m, 0, rand_field(dims, 4))
    lhs = O.vdot(xe, O.d_eo(F, L, yo))
    rhs = -O.vdot(O.d_oe(F, L, xe), yo)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # odd hops only: D maps even to odd entirely
    full = O.dslash(F, L, xe)
    assert np.abs(np.where(m, full, 0)).max() == 0.0


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 6)])
def test_dense_D_anti_hermitian(dims):
    """The assembled dense D satisfies D + D^H = 0."""
    F, L = random_links(dims)
    D = O.dense_M(F, L, 0.0)
    assert np.abs(D + D.conj().T).max() <= 1e-14 * np.abs(D).max()


def test_gauge_covariance():
    """F -> Om(x) F Om(x+mu)^H, L -> Om(x) L Om(x+3mu)^H, psi -> Om psi gives D' psi' = Om D psi.

    Catches a wrong neighbour pairing of either link (e.g. the long link paired
    with the one-hop neighbour).
    """
    dims = (4, 6, 8, 10)
    F, L = random_links(dims, seed=21)
    Om = I.random_gauge_transform(dims, 99)
    psi = rand_field(dims, 5)

    def shift(A, mu, h):
        # A(x + h mu) on the [T][Z][Y][X] grid
        axis = 3 - mu
        return np.roll(A, -h, axis=axis)

    Fp, Lp = np.empty_like(F), np.empty_like(L)
    for mu in range(4):
        Fp[mu] = Om @ F[mu] @ shift(Om, mu, 1).conj().swapaxes(-1, -2)
        Lp[mu] = Om @ L[mu] @ shift(Om, mu, 3).conj().swapaxes(-1, -2)
    psip = np.einsum("...ab,...b->...a", Om, psi)
    lhs = O.dslash(Fp, Lp, psip)
    rhs = np.einsum("...ab,...b->...a", Om, O.dslash(F, L, psi))
    assert rel(lhs, rhs) <= 1e-13


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (8, 10, 12, 16)])
def test_point_source_worked_example(dims):
    """A point source delta_{x,x0} e_c reaches exactly four sites per direction.

    At x0 - mu: F_mu(x0-mu) e_c; at x0 + mu: -F_mu(x0)^H e_c;
    at x0 - 3mu: L_mu(x0-3mu) e_c; at x0 + 3mu: -L_mu(x0)^H e_c; zero elsewhere.
    The anisotropic lattice catches axis mix-ups.
    """
    F, L = random_links(dims, seed=31)
    X, Y, Z, T = dims
    x0 = (3, 5, 7, 11 % T)
    c = 1
    src = np.zeros((T, Z, Y, X, 3), dtype=np.complex128)
    src[x0[3], x0[2], x0[1], x0[0], c] = 1.0
    out = O.dslash(F, L, src)
    expect = np.zeros_like(out)

    def at(A, xyzt):
        return A[xyzt[3], xyzt[2], xyzt[1], xyzt[0]]

    def moved(mu, h):
        x = list(x0)
        x[mu] = (x[mu] + h) % dims[mu]
        return tuple(x)

    for mu in range(4):
        for h, U in ((1, F[mu]), (3, L[mu])):
            xm, xp = moved(mu, -h), moved(mu, +h)
            at(expect, xm)[:] += at(U, xm)[:, c]
            at(expect, xp)[:] -= at(U, x0).conj()[c, :]
    assert rel(out, expect) <= 1e-15


def test_site_function_matches_full():
    dims = (4, 6, 8, 10)
    F, L = random_links(dims)
    psi = rand_field(dims, 6)
    full = O.dslash(F, L, psi)
    for s in [(0, 0, 0, 0), (3, 5, 7, 9), (1, 2, 3, 4)]:
        got = O.dslash_site(F, L, psi, s)
        assert np.array_equal(got, full[s[3], s[2], s[1], s[0]])


# ------------------------------------------------------- operator A, spectra
@pytest.mark.parametrize("dims", [(4, 4, 4, 6), (2, 2, 2, 2), (4, 6, 4, 8)])
def test_free_field_spectrum(dims):
    """spec(A) = (2m)^2 + 4 sum_mu (c1 sin p + c3 sin 3p)^2, half multiplicity."""
    F, L = free_links(dims)
    two_m = 0.1
    w = np.linalg.eigvalsh(O.dense_A(F, L, two_m))
    expect = pins.free_even_spectrum(dims, C1, C3, two_m)
    assert np.abs(np.sort(w) - expect).max() <= 1e-12


def test_normalisation_against_lambda_max():
    """Section 2 quotes lambda_max(M^H M) ~ 23 for HISQ.

    With the fat coefficient of the free HISQ action (9/8) and no factor 1/2
    in D, the free-field maximum is 16 (7/6)^2 = 21.78; with a 1/2 it would
    be 5.44.  The lattice 4^3 x 6 contains p = pi/2 in every direction.
    """
    dims = (4, 4, 4, 6)
    F, L = free_links(dims, c1=9 / 8, c3=-1 / 24)
    lmax = np.linalg.eigvalsh(O.dense_A(F, L, 0.0)).max()
    assert abs(lmax - 16 * (7 / 6) ** 2) <= 1e-12
    assert abs(lmax - 23) / 23 < 0.06


def test_A_hermitian_bounded():
    """A is Hermitian, >= (2m)^2, and <= (2m)^2 + (8(|c1|+|c3|))^2 for unitary links."""
    dims = (4, 4, 4, 6)
    F, L = random_links(dims, eps=1.0)
    two_m = 0.3
    A = O.dense_A(F, L, two_m)
    assert np.abs(A - A.conj().T).max() <= 1e-14 * np.abs(A).max()
    w = np.linalg.eigvalsh(A)
    assert w.min() >= two_m ** 2 * (1 - 1e-12)
    assert w.max() <= two_m ** 2 + (8 * (abs(C1) + abs(C3))) ** 2


def test_mass_shift_of_eigenvalues():
    """lambda(2m) = eps + (2m)^2 (Eq. (3)); the eigenvectors do not depend on m."""
    dims = (4, 4, 4, 6)
    F, L = random_links(dims)
    A0 = O.dense_A(F, L, 0.0)
    A1 = O.dense_A(F, L, 0.2)
    assert np.abs((A1 - A0) - 0.04 * np.eye(A0.shape[0])).max() <= 1e-15
    w0 = np.linalg.eigvalsh(A0)
    w1 = np.linalg.eigvalsh(A1)
    assert np.abs(w1 - (w0 + 0.04)).max() <= 1e-12


# --------------------------------------------------------- Schur and solves
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4)])
def test_schur_matches_dense_lu(dims):
    """Even-odd Schur solve + odd reconstruction equals dense LU of M = D + 2m."""
    F, L = random_links(dims, seed=41)
    two_m = 0.2
    eta = rand_field(dims, 7)
    M = O.dense_M(F, L, two_m)
    psi_lu = np.linalg.solve(M, eta.reshape(-1)).reshape(eta.shape)
    y_e = O.source_even(F, L, two_m, eta)
    psi_e, iters, res = O.solve_even(F, L, two_m, y_e, tol=1e-14)
    assert res <= 1e-14
    psi_o = O.reconstruct_odd(F, L, two_m, psi_e, eta)
    psi = psi_e + psi_o
    assert rel(psi, psi_lu) <= 1e-12
    # the reconstruction makes the odd rows of M psi = eta exact
    m = O.even_mask(dims)[..., None]
    r = O.apply_M(F, L, two_m, psi) - eta
    assert np.abs(np.where(m, 0, r)).max() <= 1e-12 * np.abs(eta).max()


def test_full_normal_equation_matches_schur():
    """CG on the full normal equation M^H M psi = M^H eta (Eq. (1)) equals Schur + reconstruction."""
    dims = (4, 4, 4, 6)
    F, L = random_links(dims, seed=43)
    two_m = 0.3
    eta = rand_field(dims, 8)
    b = O.apply_Mdag(F, L, two_m, eta)
    psi_full, _, res = O.cg(lambda v: O.apply_Mdag(F, L, two_m, O.apply_M(F, L, two_m, v)),
                            b, tol=1e-13)
    assert res <= 1e-13
    y_e = O.source_even(F, L, two_m, eta)
    psi_e, _, _ = O.solve_even(F, L, two_m, y_e, tol=1e-13)
    psi = psi_e + O.reconstruct_odd(F, L, two_m, psi_e, eta)
    assert rel(psi_full, psi) <= 1e-11


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (6, 4, 8, 6)])
def test_free_field_cg_matches_fft(dims):
    """Free field: the oracle CG solution equals the FFT solution of ((2m)^2 - D^2) psi = y."""
    F, L = free_links(dims)
    two_m = 0.05
    m = O.even_mask(dims)[..., None]
    y = np.where(m, rand_field(dims, 9), 0)
    psi, iters, res = O.solve_even(F, L, two_m, y, tol=1e-13)
    assert res <= 1e-13
    ref = pins.free_solve_fft(dims, C1, C3, two_m, y)
    assert np.abs(np.where(m, 0, ref)).max() <= 1e-12 * np.abs(ref).max()
    assert rel(psi, ref) <= 1e-11


def test_cg_edge_cases():
    dims = (4, 4, 4, 4)
    F, L = random_links(dims)
    two_m = 0.2
    m = O.even_mask(dims)[..., None]
    # b = 0: x = 0, no iterations
    b0 = np.zeros((4, 4, 4, 4, 3), dtype=np.complex128)
    x, it, res = O.solve_even(F, L, two_m, b0)
    assert it == 0 and not x.any()
    # exact initial guess: no iterations
    b = np.where(m, rand_field(dims, 10), 0)
    A = O.dense_A(F, L, two_m)
    xc = np.linalg.solve(A, O.to_compact(b, dims))
    x, it, res = O.solve_even(F, L, two_m, b, x0=O.from_compact(xc, dims), tol=1e-10)
    assert it == 0 and res <= 1e-10
    # max_iter reached: returns the current iterate
    x, it, res = O.solve_even(F, L, two_m, b, tol=1e-14, max_iter=3)
    assert it == 3 and res > 1e-14


def test_cg_iteration_count_tracks_condition_number():
    """CG work grows as the mass falls (section 2: kappa ~ lambda_max/(2m)^2)."""
    dims = (4, 4, 4, 8)
    F, L = random_links(dims, eps=0.3)
    m = O.even_mask(dims)[..., None]
    b = np.where(m, rand_field(dims, 12), 0)
    its = [O.solve_even(F, L, tm, b, tol=1e-10)[1] for tm in (0.5, 0.1, 0.02)]
    assert its[0] < its[1] < its[2]


# ---------------------------------------------------- eigenpairs, deflation
def test_arpack_matches_dense():
    dims = (4, 4, 4, 6)
    F, L = random_links(dims, seed=51)
    w_d, V_d = O.lowest_eigenpairs(F, L, 0.1, 12, method="dense")
    w_a, V_a = O.lowest_eigenpairs(F, L, 0.1, 12, method="arpack",
                                   v0=np.ones(V_d.shape[0], dtype=np.complex128))
    assert np.abs(w_a - w_d).max() <= 1e-12 * w_d.max()
    assert np.abs(V_a.conj().T @ V_a - np.eye(12)).max() <= 1e-12
    # same subspace: projectors agree
    Pd = V_d @ V_d.conj().T
    Pa = V_a @ V_a.conj().T
    assert np.abs(Pd - Pa).max() <= 1e-8


def test_free_field_lowest_modes():
    dims = (4, 4, 4, 8)
    F, L = free_links(dims)
    expect = pins.free_even_spectrum(dims, C1, C3, 0.1)
    w, V = O.lowest_eigenpairs(F, L, 0.1, 24, method="dense")
    assert np.abs(w - expect[:24]).max() <= 1e-12


def test_deflation_special_cases():
    """Eq. (4): with exact eigenvectors, b in span(V) gives x0 = A^{-1} b and CG does no work;
    for a general b the residual b - A x0 has no component along V."""
    dims = (4, 4, 4, 6)
    F, L = random_links(dims, seed=61)
    two_m = 0.1
    k = 16
    w, V = O.lowest_eigenpairs(F, L, two_m, k, method="dense")
    A = O.dense_A(F, L, two_m)
    coef = I.gaussian_even_vectors(1, k, 5)[0]
    b = V @ coef
    x0 = O.deflation_guess(V, w, b)
    assert rel(A @ x0, b) <= 1e-12
    bf = O.from_compact(b, dims)
    x, it, res = O.solve_even(F, L, two_m, bf, x0=O.from_compact(x0, dims), tol=1e-10)
    assert it == 0
    g = I.gaussian_even_vectors(1, V.shape[0], 6)[0]
    x0 = O.deflation_guess(V, w, g)
    assert np.abs(V.conj().T @ (g - A @ x0)).max() <= 1e-12 * np.linalg.norm(g)
    # the mass-independent form: eigenvalues of A(0) shifted by (2m)^2
    w0, V0 = O.lowest_eigenpairs(F, L, 0.0, k, method="dense")
    x0b = O.deflation_guess(V0, w0 + two_m ** 2, g)
    assert rel(x0b, x0) <= 1e-10


def test_deflation_reduces_iterations():
    """Deflation helps far more at light mass than at heavy mass (Table 2)."""
    dims = (4, 4, 4, 8)
    F, L = random_links(dims, eps=0.3, seed=71)
    m = O.even_mask(dims)[..., None]
    b = np.where(m, rand_field(dims, 13), 0)
    w0, V = O.lowest_eigenpairs(F, L, 0.0, 48, method="dense")
    gains = []
    for tm in (0.5, 0.01):
        _, it_plain, _ = O.solve_even(F, L, tm, b, tol=1e-10)
        x0 = O.from_compact(O.deflation_guess(V, w0 + tm * tm, O.to_compact(b, dims)), dims)
        _, it_defl, res = O.solve_even(F, L, tm, b, x0=x0, tol=1e-10)
        assert res <= 1e-10
        gains.append(it_plain / max(it_defl, 1))
    assert gains[1] > gains[0]
