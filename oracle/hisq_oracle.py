"""Oracle: a plain, slow FP64 CPU statement of what the HISQ solve path computes.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this module.  It shares no code with
the GPU library; both read the same seeded inputs from
`paper_2502_00152_amd.inputs`, which holds none of the method's arithmetic.

What is computed, and where the paper defines it (arXiv:2502.00152):

* The quark matrix M = D + 2m, D anti-Hermitian (section 2, before Eq. (1)).
  The stencil D itself (fat one-hop + Naik three-hop) is in hisq_stencil.c.
* Staggered phases and the antiperiodic time boundary are folded into the
  links here (`fold_links`); the paper only names HISQ, so the conventions are
  readings (listed in the design notes): eta_0 = 1, eta_1 = (-1)^x,
  eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z); a hop of length h in time from t
  carries (-1)^floor((t+h)/T).
* The normal equation M^H M psi = M^H eta (Eq. (1)) solved by even-odd
  (Schur) preconditioning (section 2, the MILC/QUDA workflow paragraph):
  y = M^H eta, even-site system A psi_e = y_e with
  A = (2m)^2 - D_eo D_oe, then the odd half from the odd rows of M psi = eta,
  psi_o = (eta_o - D_oe psi_e) / (2m).  The printed odd formula is garbled;
  this is the reading that makes M psi = eta hold.
* CG with a true-residual stopping test (section 2, the sentence after Eq. (1)
  defines the stopping criterion as a true residual).
* The low modes of A (Eqs. (2)-(3): lambda = eps + (2m)^2 with eps the
  eigenvalues of the massless squared operator) by dense Hermitian
  eigendecomposition or ARPACK; the paper's thick-restart Lanczos is one way
  to reach them and is not restated here.
* The deflation initial guess x0 = sum_i v_i v_i^H b / lambda_i (Eq. (4)).

Vectors are canonical complex128 arrays [T][Z][Y][X][3] (x fastest); an
"even-site vector" is such an array that is zero on odd sites.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libhisq_oracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_dslash.argtypes = [P, P, P, P, P, ctypes.c_int, ctypes.c_int]
        lib.oracle_dslash.restype = None
        lib.oracle_dslash_site.argtypes = [P, P, P, P, ctypes.c_int64, P]
        lib.oracle_dslash_site.restype = None
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def n_threads() -> int:
    v = os.environ.get("ORACLE_THREADS") or os.environ.get("OMP_NUM_THREADS")
    return int(v) if v else (os.cpu_count() or 1)


def _dims_arr(dims):
    return (ctypes.c_int * 4)(*[int(d) for d in dims])


def dims_of(field: np.ndarray):
    """(X, Y, Z, T) of a canonical field [T][Z][Y][X][3] or links [4][T][Z][Y][X][3][3]."""
    if field.ndim == 7:
        _, T, Z, Y, X = field.shape[:5]
    else:
        T, Z, Y, X = field.shape[-5:-1]
    return (X, Y, Z, T)


# --------------------------------------------------------------------------
# Lattice geometry (readings of the conventions the paper leaves implicit)
# --------------------------------------------------------------------------
def coordinates(dims):
    """Integer coordinate arrays x, y, z, t, each shaped [T][Z][Y][X]."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    return x, y, z, t


def parity(dims) -> np.ndarray:
    x, y, z, t = coordinates(dims)
    return (x + y + z + t) % 2


def even_mask(dims) -> np.ndarray:
    return parity(dims) == 0


def staggered_eta(dims, mu: int) -> np.ndarray:
    """eta_mu(x): 1, (-1)^x, (-1)^(x+y), (-1)^(x+y+z) for mu = 0..3."""
    x, y, z, t = coordinates(dims)
    s = [np.zeros_like(x), x, x + y, x + y + z][mu]
    return np.where(s % 2 == 0, 1.0, -1.0)


def time_boundary_sign(dims, hop: int) -> np.ndarray:
    """(-1)^floor((t+hop)/T): the antiperiodic sign of a time hop from t."""
    x, y, z, t = coordinates(dims)
    T = dims[3]
    return np.where(((t + hop) // T) % 2 == 0, 1.0, -1.0)


def fold_links(W, N, c_fat: float, c_long: float, phases: bool = True,
               antiperiodic: bool = True):
    """F_mu = eta_mu s1_mu c_fat W_mu and L_mu = eta_mu s3_mu c_long N_mu."""
    dims = dims_of(W)
    F = np.array(W, dtype=np.complex128) * c_fat
    L = np.array(N, dtype=np.complex128) * c_long
    for mu in range(4):
        s1 = np.ones(dims[::-1])
        s3 = np.ones(dims[::-1])
        if phases:
            e = staggered_eta(dims, mu)
            s1 = s1 * e
            s3 = s3 * e
        if antiperiodic and mu == 3:
            s1 = s1 * time_boundary_sign(dims, 1)
            s3 = s3 * time_boundary_sign(dims, 3)
        F[mu] *= s1[..., None, None]
        L[mu] *= s3[..., None, None]
    return F, L


# --------------------------------------------------------------------------
# The stencil and the Schur pieces
# --------------------------------------------------------------------------
ROWS_EVEN, ROWS_ODD, ROWS_ALL = 0, 1, 2


def dslash(F, L, psi, rows: int = ROWS_ALL) -> np.ndarray:
    """D psi (C stencil) on the selected rows; other rows are zero."""
    lib = _load()
    dims = dims_of(F)
    F = np.ascontiguousarray(F, dtype=np.complex128)
    L = np.ascontiguousarray(L, dtype=np.complex128)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    lib.oracle_dslash(_dims_arr(dims), F.ctypes.data, L.ctypes.data, psi.ctypes.data,
                      out.ctypes.data, int(rows), n_threads())
    return out


def dslash_site(F, L, psi, site_xyzt) -> np.ndarray:
    """(D psi)(x) at one site, computed on its own (for sampled checks)."""
    lib = _load()
    dims = dims_of(F)
    x, y, z, t = site_xyzt
    lex = ((t * dims[2] + z) * dims[1] + y) * dims[0] + x
    out = np.zeros(3, dtype=np.complex128)
    lib.oracle_dslash_site(_dims_arr(dims), F.ctypes.data, L.ctypes.data, psi.ctypes.data,
                           int(lex), out.ctypes.data)
    return out


def d_eo(F, L, v_odd):
    """D_eo: odd sites -> even sites."""
    return dslash(F, L, v_odd, ROWS_EVEN)


def d_oe(F, L, v_even):
    """D_oe: even sites -> odd sites."""
    return dslash(F, L, v_even, ROWS_ODD)


def apply_A(F, L, two_m: float, v_even):
    """A v = (2m)^2 v - D_eo D_oe v on even-site vectors."""
    return (two_m * two_m) * v_even - d_eo(F, L, d_oe(F, L, v_even))


def apply_M(F, L, two_m: float, psi):
    """M psi = D psi + 2m psi on the full lattice."""
    return dslash(F, L, psi, ROWS_ALL) + two_m * psi


def apply_Mdag(F, L, two_m: float, psi):
    """M^H psi = -D psi + 2m psi (D is anti-Hermitian)."""
    return -dslash(F, L, psi, ROWS_ALL) + two_m * psi


def source_even(F, L, two_m: float, eta):
    """y_e = (M^H eta)_e = 2m eta_e - D_eo eta_o."""
    mask = even_mask(dims_of(F))[..., None]
    eta_e = np.where(mask, eta, 0)
    eta_o = np.where(mask, 0, eta)
    return two_m * eta_e - d_eo(F, L, eta_o)


def reconstruct_odd(F, L, two_m: float, psi_e, eta):
    """psi_o = (eta_o - D_oe psi_e) / (2m), from the odd rows of M psi = eta."""
    mask = even_mask(dims_of(F))[..., None]
    eta_o = np.where(mask, 0, eta)
    return (eta_o - d_oe(F, L, psi_e)) / two_m


# --------------------------------------------------------------------------
# CG with a true-residual stopping test
# --------------------------------------------------------------------------
def vdot(u, v) -> complex:
    """<u, v> = sum conj(u) v."""
    return complex(np.vdot(u.ravel(), v.ravel()))


def norm(u) -> float:
    return float(np.sqrt(vdot(u, u).real))


def cg(apply, b, x0=None, tol: float = 1e-10, max_iter: int = 100000, history=None):
    """Conjugate gradient on a Hermitian positive definite operator.

    Stops when the true residual ||b - A x|| / ||b|| <= tol.  The iterated
    residual decides when to recompute the true one; if the true one fails the
    test, iteration continues from it with the search direction kept.
    Returns (x, iterations, true relative residual).  Iterations count the
    operator applications inside the loop (not the initial residual nor the
    true-residual recomputations).
    """
    bnorm = norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - apply(x)
    rho = vdot(r, r).real
    if np.sqrt(rho) <= tol * bnorm:
        return x, 0, np.sqrt(rho) / bnorm
    p = r.copy()
    k = 0
    while k < max_iter:
        q = apply(p)
        alpha = rho / vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        rho_new = vdot(r, r).real
        k += 1
        if history is not None:
            history.append(np.sqrt(rho_new) / bnorm)
        if np.sqrt(rho_new) <= tol * bnorm:
            r = b - apply(x)
            rho_new = vdot(r, r).real
            if np.sqrt(rho_new) <= tol * bnorm:
                rho = rho_new
                break
        beta = rho_new / rho
        rho = rho_new
        p = r + beta * p
    true_rel = norm(b - apply(x)) / bnorm
    return x, k, true_rel


def solve_even(F, L, two_m, y_e, x0=None, tol=1e-10, max_iter=100000):
    """psi_e = A^{-1} y_e by CG (the paper's 'CG' baseline)."""
    return cg(lambda v: apply_A(F, L, two_m, v), y_e, x0=x0, tol=tol, max_iter=max_iter)


# --------------------------------------------------------------------------
# Compact even-site vectors, dense operators and eigenpairs
# --------------------------------------------------------------------------
def to_compact(v, dims):
    """Even-site entries of a full-lattice vector, in lexicographic order."""
    return v[even_mask(dims)].reshape(-1)


def from_compact(c, dims):
    X, Y, Z, T = dims
    out = np.zeros((T, Z, Y, X, 3), dtype=np.complex128)
    out[even_mask(dims)] = c.reshape(-1, 3)
    return out


def dense_A(F, L, two_m):
    """A assembled column by column on the compact even-site basis."""
    dims = dims_of(F)
    n = 3 * int(even_mask(dims).sum())
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        A[:, j] = to_compact(apply_A(F, L, two_m, from_compact(e, dims)), dims)
    return A


def dense_M(F, L, two_m):
    """The full-lattice M = D + 2m, assembled column by column (canonical order)."""
    dims = dims_of(F)
    X, Y, Z, T = dims
    n = 3 * X * Y * Z * T
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((T, Z, Y, X, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for j in range(n):
        flat[:] = 0
        flat[j] = 1
        M[:, j] = apply_M(F, L, two_m, e).reshape(-1)
    return M


def lowest_eigenpairs(F, L, two_m, k, method="auto", tol=1e-13, v0=None):
    """The k smallest eigenpairs of A (ascending), vectors as compact columns.

    method 'dense' uses numpy.linalg.eigh on the assembled A; 'arpack' uses
    scipy.sparse.linalg.eigsh with the oracle's A as a linear operator.
    """
    dims = dims_of(F)
    n = 3 * int(even_mask(dims).sum())
    if method == "auto":
        method = "dense" if n <= 2000 else "arpack"
    if method == "dense":
        w, V = np.linalg.eigh(dense_A(F, L, two_m))
        return w[:k], V[:, :k]
    from scipy.sparse.linalg import LinearOperator, eigsh

    def mv(c):
        return to_compact(apply_A(F, L, two_m, from_compact(np.asarray(c).reshape(-1), dims)),
                          dims)

    op = LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    w, V = eigsh(op, k=k, which="SA", tol=tol, v0=v0, ncv=max(2 * k + 1, 20))
    order = np.argsort(w)
    return w[order], V[:, order]


def deflation_guess(V, evals, b):
    """x0 = sum_i v_i (1/lambda_i) v_i^H b, Eq. (4); V columns orthonormal."""
    lam = np.asarray(evals, dtype=np.float64)
    c = V.conj().T @ b
    c = c / (lam[:, None] if c.ndim == 2 else lam)
    return V @ c
