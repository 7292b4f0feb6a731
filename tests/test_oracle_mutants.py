"""Plant plausible mistakes in a copy of the oracle and check that the pins catch them.

Each mutant is a text edit of the oracle's C stencil (or of its link folding),
compiled into a temporary library on the CPU; the pins of test_oracle_pins
must then fail.  This shows that the pins constrain the oracle rather than
restate it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import hisq_oracle as O
from paper_2502_00152_amd import inputs as I
from tests import pins

SRC = os.path.join(os.path.dirname(O.__file__), "hisq_stencil.c")

MUTANTS = {
    # backward hop reads the link at x instead of x - h mu
    "backward_link_site": ("adj_mul_sub(links[h] + lb * 9", "adj_mul_sub(links[h] + lex * 9"),
    # backward hop uses the transpose instead of the adjoint
    "transpose_not_adjoint": ("conj(U[3 * b + a])", "U[3 * b + a]"),
    # Naik term hops two sites instead of three
    "naik_hop_length": ("const int hops[2] = {1, 3};", "const int hops[2] = {1, 2};"),
    # forward hop multiplies by U^T
    "forward_transposed": ("acc[a] += U[3 * a + b] * v[b];", "acc[a] += U[3 * b + a] * v[b];"),
    # backward sign flipped (D no longer anti-Hermitian)
    "backward_sign": ("acc[a] -= conj(U[3 * b + a]) * v[b];", "acc[a] += conj(U[3 * b + a]) * v[b];"),
}


def _build_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-fcx-limited-range", "-fopenmp", "-fPIC",
                    "-shared", "-o", str(lib), str(path)], check=True)
    L = ctypes.CDLL(str(lib))
    P = ctypes.c_void_p
    L.oracle_dslash.argtypes = [P, P, P, P, P, ctypes.c_int, ctypes.c_int]
    L.oracle_dslash_site.argtypes = [P, P, P, P, ctypes.c_int64, P]
    L.oracle_max_threads.restype = ctypes.c_int
    return L


def _pins_hold() -> bool:
    """The stencil pins, compactly: anti-Hermiticity, covariance-free spectrum."""
    dims = (4, 4, 4, 6)
    W = I.random_su3_field(dims, 0.5, 11)
    N = I.random_su3_field(dims, 0.5, 12)
    F, L = O.fold_links(W, N, I.C_FAT, I.C_LONG)
    x, y = I.gaussian_source(dims, 1), I.gaussian_source(dims, 2)
    lhs = O.vdot(x, O.dslash(F, L, y))
    rhs = -O.vdot(O.dslash(F, L, x), y)
    anti = abs(lhs - rhs) <= 1e-13 * abs(lhs)
    U = I.unit_links(dims)
    Ff, Lf = O.fold_links(U, U, I.C_FAT, I.C_LONG)
    w = np.linalg.eigvalsh(O.dense_A(Ff, Lf, 0.1))
    A = O.dense_A(Ff, Lf, 0.1)
    herm = np.abs(A - A.conj().T).max() <= 1e-12
    spec = herm and np.abs(np.sort(w) - pins.free_even_spectrum(dims, I.C_FAT, I.C_LONG, 0.1)).max() <= 1e-10
    return bool(anti and spec)


def test_unmutated_oracle_passes():
    assert _pins_hold()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_stencil_mutant_is_caught(tmp_path, monkeypatch, name):
    monkeypatch.setattr(O, "_lib", _build_mutant(tmp_path, name))
    assert not _pins_hold()


@pytest.mark.parametrize("mistake", ["no_time_sign_on_naik", "eta_t_wrong", "c3_sign"])
def test_folding_mutant_is_caught(monkeypatch, mistake):
    real_fold = O.fold_links

    if mistake == "no_time_sign_on_naik":
        def tsign(dims, hop, _orig=O.time_boundary_sign):
            return _orig(dims, 1)
        monkeypatch.setattr(O, "time_boundary_sign", tsign)
    elif mistake == "eta_t_wrong":
        def eta(dims, mu, _orig=O.staggered_eta):
            return _orig(dims, 2 if mu == 3 else mu)
        monkeypatch.setattr(O, "staggered_eta", eta)
    else:
        monkeypatch.setattr(O, "fold_links",
                            lambda W, N, c1, c3, **k: real_fold(W, N, c1, -c3, **k))
    assert not _pins_hold()
