"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no staggered phases, no boundary signs, no stencil, no
solver).  Both sides of every parity check read the fields produced here.

Gauge fields
    Each link is a random SU(3) matrix W = exp(i*eps*H) with H a traceless
    Hermitian 3x3 matrix, H = sum_a h_a * lambda_a / 2 over the eight
    Gell-Mann matrices, h_a ~ N(0, 1) i.i.d.  The exponential is evaluated from
    the eigendecomposition of H, H = Q diag(theta) Q^H, as
    W = Q diag(exp(i*eps*theta)) Q^H.  Fat and long (Naik) links are two
    independent draws from this distribution, with their own seeds.  The paper
    measures on MILC HISQ ensembles (Table 1), which are not available; these
    fields stand in for them at the paper's shapes.

Layouts (canonical, lexicographic with x fastest)
    dims = (X, Y, Z, T)
    links   complex128 [4][T][Z][Y][X][3][3]   (mu = x, y, z, t; row-major a,b)
    spinors complex128 [nrhs][T][Z][Y][X][3]

Random streams
    numpy PCG64.  Links are drawn direction by direction and time slice by time
    slice, in that order, from one generator per field; a source is one
    generator per right-hand side.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "GELL_MANN",
    "random_su3_field",
    "random_su3_matrices",
    "gaussian_source",
    "gaussian_even_vectors",
    "random_gauge_transform",
    "unit_links",
    "workload",
    "WORKLOADS",
    "random_su3_field_device",
]


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


GELL_MANN = _gell_mann()


def random_su3_matrices(rng: np.random.Generator, shape, eps: float) -> np.ndarray:
    """Draw exp(i*eps*H) for a batch of Gaussian traceless Hermitian H."""
    n = int(np.prod(shape))
    h = rng.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", h, GELL_MANN) * 0.5
    theta, Q = np.linalg.eigh(H)
    ph = np.exp(1j * eps * theta)
    W = np.einsum("nij,nj,nkj->nik", Q, ph, Q.conj())
    return W.reshape(tuple(shape) + (3, 3))


def random_su3_field(dims, eps: float, seed: int) -> np.ndarray:
    """Links complex128 [4][T][Z][Y][X][3][3], one PCG64 stream per field."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((4, T, Z, Y, X, 3, 3), dtype=np.complex128)
    for mu in range(4):
        for t in range(T):
            out[mu, t] = random_su3_matrices(rng, (Z, Y, X), eps)
    return out


def unit_links(dims) -> np.ndarray:
    """Free field: every link the 3x3 identity."""
    X, Y, Z, T = (int(d) for d in dims)
    out = np.zeros((4, T, Z, Y, X, 3, 3), dtype=np.complex128)
    for a in range(3):
        out[..., a, a] = 1.0
    return out


def gaussian_source(dims, seed: int) -> np.ndarray:
    """Full-lattice source complex128 [T][Z][Y][X][3], Re and Im ~ N(0,1)."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((T, Z, Y, X, 3))
    im = rng.standard_normal((T, Z, Y, X, 3))
    return re + 1j * im


def gaussian_even_vectors(n: int, n_cplx: int, seed: int) -> np.ndarray:
    """n generic complex vectors of length n_cplx (no lattice structure)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n, n_cplx)) + 1j * rng.standard_normal((n, n_cplx))


def random_gauge_transform(dims, seed: int, eps: float = 3.0) -> np.ndarray:
    """Site-local SU(3) matrices Omega(x), complex128 [T][Z][Y][X][3][3]."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    return random_su3_matrices(rng, (T, Z, Y, X), eps)


# Synthetic workloads at the paper's shapes.  Seeds: fat 10000c+1,
# long 10000c+2, source j 10000c+100+j, eigensolver start 10000c+7.
WORKLOADS = {
    0: dict(name="plain-cg-8^4", dims=(8, 8, 8, 8), eps=0.3, two_m=0.1, nrhs=1,
            n_ev=0, tol=1e-10),
    1: dict(name="deflated-cg-16^3x32", dims=(16, 16, 16, 32), eps=0.5, two_m=0.01,
            nrhs=12, n_ev=64, tol=1e-10),
    2: dict(name="mixed-precision-32^3x64", dims=(32, 32, 32, 64), eps=0.5,
            two_m=0.005, nrhs=24, n_ev=256, tol=1e-10),
    # one GPU's share of a large-lattice solve with the learned guess; 128
    # eigenpairs and 48 streamed training pairs keep a run within minutes
    # (512 pairs fit one GPU's memory with one FP64 Lanczos basis, about 180
    # GB, but their eigensolve takes far longer than a benchmark run)
    4: dict(name="learned-guess-48^3x96", dims=(48, 48, 48, 96), eps=0.5, two_m=0.002,
            nrhs=12, n_ev=128, tol=1e-10, n_pairs=48),
}
C_FAT = 1.0
C_LONG = -1.0 / 24.0

# Uneven batch: four lattices x three masses, fewer RHS on larger lattices.
# Seeds of lattice l: fat 30000+1000l+1, long +2, source j of mass k
# 30000+1000l+100+10k+j.
UNEVEN_BATCH = dict(name="uneven-batch", eps=0.3, masses=(0.1, 0.02, 0.005), tol=1e-10,
                    lattices=(((8, 8, 8, 8), 32), ((12, 12, 12, 12), 16),
                              ((16, 16, 16, 32), 8), ((24, 24, 24, 48), 4)))


def workload(c: int) -> dict:
    """Recipe of workload c, with its seeds."""
    d = dict(WORKLOADS[c])
    d["seed_fat"] = 10000 * c + 1
    d["seed_long"] = 10000 * c + 2
    d["seed_src"] = [10000 * c + 100 + j for j in range(d["nrhs"])]
    d["seed_eig"] = 10000 * c + 7
    d["c_fat"] = C_FAT
    d["c_long"] = C_LONG
    return d


def random_su3_field_device(dims, eps: float, seed: int, device="cuda"):
    """Same distribution as random_su3_field, drawn with torch on the device.

    For lattices too large to draw on the host quickly (32^3 x 64: a minute per
    field); the random stream differs from random_su3_field.  Parity tests at
    such sizes copy these links to the host for the oracle.
    exp(i eps H) is evaluated by scaling and squaring of its Taylor series
    (||i eps H / 16|| < 0.4 for the eps used here, 14 terms: error < 1e-16).
    """
    import torch

    X, Y, Z, T = (int(d) for d in dims)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    lam = torch.from_numpy(np.ascontiguousarray(GELL_MANN.reshape(8, 9))).to(device)
    out = torch.empty((4, T, Z, Y, X, 3, 3), dtype=torch.complex128, device=device)
    eye = torch.eye(3, dtype=torch.complex128, device=device)
    for mu in range(4):
        h = torch.randn((T, Z, Y, X, 8), dtype=torch.float64, generator=gen, device=device)
        H = (torch.matmul(h.to(torch.complex128), lam) * 0.5).reshape(T, Z, Y, X, 3, 3)
        B = (1j * eps / 16.0) * H
        E = eye.expand_as(B).clone()
        term = eye.expand_as(B).clone()
        for k in range(1, 15):
            term = torch.matmul(term, B) / k
            E = E + term
        for _ in range(4):
            E = torch.matmul(E, E)
        out[mu] = E
    return out


def nn_initial_params(seed: int, channels: int = 8) -> np.ndarray:
    """Initial parameters of the learned-guess network, float32, in the order
    W1 [9][C][1], W2 [9][C][C], W3 [9][1][C], g1 [C][2], g2 [C][2]: Gaussian
    weights scaled by 1/sqrt(9 fan_in), gates (a, b) = (0, 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    C = channels
    parts = [rng.standard_normal(9 * C * 1) / np.sqrt(9 * 1),
             rng.standard_normal(9 * C * C) / np.sqrt(9 * C),
             rng.standard_normal(9 * 1 * C) / np.sqrt(9 * C)]
    g = np.zeros((C, 2))
    g[:, 1] = 2.0
    parts += [g.ravel(), g.ravel()]
    return np.concatenate(parts).astype(np.float32)
