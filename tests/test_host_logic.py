"""Host logic of the library tested on the CPU: the dense Hermitian Jacobi
eigensolver used for the small projected matrices of the eigensolver."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def heev(tmp_path_factory):
    out = tmp_path_factory.mktemp("hostlib") / "libhost_eig_test.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(out),
                    os.path.join(ROOT, "paper_2502_00152_amd", "csrc", "dense_eig.cpp"),
                    os.path.join(ROOT, "tests", "host_eig_shim.cpp")], check=True)
    L = ctypes.CDLL(str(out))
    L.test_heev.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_int]
    L.test_heev.restype = ctypes.c_int

    def run(A):
        n = A.shape[0]
        a = np.ascontiguousarray(A, dtype=np.complex128).copy()
        w = np.zeros(n)
        Z = np.zeros((n, n), dtype=np.complex128)
        sweeps = L.test_heev(n, a.ctypes.data, w.ctypes.data, Z.ctypes.data, 60)
        return sweeps, w, Z
    return run


@pytest.mark.parametrize("n", [1, 2, 5, 33, 96])
def test_jacobi_hermitian(heev, n):
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = M + M.conj().T
    sweeps, w, Z = heev(A)
    assert sweeps >= 0
    ref = np.linalg.eigvalsh(A)
    assert np.abs(w - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(Z.conj().T @ Z - np.eye(n)).max() <= 1e-12
    assert np.abs(A @ Z - Z * w).max() <= 1e-11 * np.abs(ref).max()


def test_jacobi_graded_arrowhead(heev):
    """The filtered Lanczos matrices span many orders of magnitude."""
    n = 60
    rng = np.random.default_rng(1)
    d = np.concatenate([10.0 ** rng.uniform(0, 12, 20), rng.uniform(-1, 1, 40)])
    A = np.diag(d).astype(np.complex128)
    A[:20, 20] = A[20, :20] = rng.standard_normal(20) * 1e-3
    for j in range(20, n - 1):
        A[j, j + 1] = A[j + 1, j] = rng.uniform(0.1, 1)
    sweeps, w, Z = heev(A)
    ref = np.linalg.eigvalsh(A)
    # backward stable: errors of order eps * ||A|| (both solvers)
    assert np.abs(w - ref).max() <= 1e-14 * np.abs(ref).max()
    assert np.abs(A @ Z - Z * w).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(Z.conj().T @ Z - np.eye(n)).max() <= 1e-12


def test_jacobi_degenerate_and_zero(heev):
    A = np.diag([2.0, 2.0, 2.0, -1.0]).astype(np.complex128)
    sweeps, w, Z = heev(A)
    assert np.allclose(w, [-1, 2, 2, 2])
    sweeps, w, Z = heev(np.zeros((3, 3), dtype=np.complex128))
    assert np.all(w == 0)


@pytest.fixture(scope="module")
def syev(tmp_path_factory):
    out = tmp_path_factory.mktemp("hostlib2") / "libhost_syev_test.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(out),
                    os.path.join(ROOT, "paper_2502_00152_amd", "csrc", "dense_eig.cpp"),
                    os.path.join(ROOT, "tests", "host_eig_shim.cpp")], check=True)
    L = ctypes.CDLL(str(out))
    L.test_syev.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.test_syev.restype = ctypes.c_int

    def run(A):
        n = A.shape[0]
        a = np.ascontiguousarray(A, dtype=np.float64).copy()
        w = np.zeros(n)
        Z = np.zeros((n, n))
        steps = L.test_syev(n, a.ctypes.data, w.ctypes.data, Z.ctypes.data)
        return steps, w, Z
    return run


def check_eig(A, steps, w, Z, rel):
    n = A.shape[0]
    assert steps >= 0
    ref = np.linalg.eigvalsh(A)
    s = max(np.abs(ref).max(), 1e-300)
    assert np.abs(w - ref).max() <= rel * s
    assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-12 * max(1, n / 50)
    assert np.abs(A @ Z - Z * w).max() <= rel * 10 * s


@pytest.mark.parametrize("n", [1, 2, 3, 7, 40, 200])
def test_qr_symmetric_dense(syev, n):
    rng = np.random.default_rng(100 + n)
    M = rng.standard_normal((n, n))
    A = M + M.T
    check_eig(A, *syev(A), rel=1e-13)


def test_qr_graded_arrowhead_tridiagonal(syev):
    """The shape of a thick-restart Lanczos matrix: kept Ritz values on the
    diagonal spanning many orders of magnitude, an arrow row/column of
    couplings, then a tridiagonal block."""
    n, k0 = 120, 40
    rng = np.random.default_rng(7)
    A = np.zeros((n, n))
    A[np.arange(k0), np.arange(k0)] = 10.0 ** rng.uniform(0, 12, k0)
    A[:k0, k0] = A[k0, :k0] = rng.standard_normal(k0) * 1e-2
    d = rng.uniform(-1, 1, n - k0)
    A[np.arange(k0, n), np.arange(k0, n)] = d
    for j in range(k0, n - 1):
        A[j, j + 1] = A[j + 1, j] = rng.uniform(0.1, 1)
    steps, w, Z = syev(A)
    check_eig(A, steps, w, Z, rel=1e-13)
    # the large (wanted) eigenvalues are accurate relative to themselves
    ref = np.linalg.eigvalsh(A)
    big = ref > 1e3
    assert np.abs(w[big] - ref[big]).max() <= 1e-12 * ref[big].max()


def test_qr_degenerate_diagonal_and_zero(syev):
    A = np.diag([2.0, 2.0, 2.0, -1.0])
    steps, w, Z = syev(A)
    assert np.allclose(w, [-1, 2, 2, 2]) and np.allclose(np.abs(Z.T @ Z), np.eye(4))
    steps, w, Z = syev(np.zeros((3, 3)))
    assert np.all(w == 0)
    # Wilkinson's matrix W21+: pairs of nearly equal eigenvalues
    n = 21
    A = np.diag(np.abs(np.arange(n) - 10.0)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    check_eig(A, *syev(A), rel=1e-13)


@pytest.fixture(scope="module")
def heev_qr(tmp_path_factory):
    out = tmp_path_factory.mktemp("hostlib3") / "libhost_heev_qr_test.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", str(out),
                    os.path.join(ROOT, "paper_2502_00152_amd", "csrc", "dense_eig.cpp"),
                    os.path.join(ROOT, "tests", "host_eig_shim.cpp")], check=True)
    L = ctypes.CDLL(str(out))
    L.test_heev_qr.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.test_heev_qr.restype = ctypes.c_int

    def run(A):
        n = A.shape[0]
        a = np.ascontiguousarray(A, dtype=np.complex128).copy()
        w = np.zeros(n)
        Z = np.zeros((n, n), dtype=np.complex128)
        steps = L.test_heev_qr(n, a.ctypes.data, w.ctypes.data, Z.ctypes.data)
        return steps, w, Z
    return run


def check_heig(A, steps, w, Z, rel):
    n = A.shape[0]
    assert steps >= 0
    ref = np.linalg.eigvalsh(A)
    s = max(np.abs(ref).max(), 1e-300)
    assert np.abs(w - ref).max() <= rel * s
    assert np.abs(Z.conj().T @ Z - np.eye(n)).max() <= 1e-12 * max(1, n / 50)
    assert np.abs(A @ Z - Z * w).max() <= rel * 10 * s


@pytest.mark.parametrize("n", [1, 2, 3, 7, 40, 200])
def test_complex_qr_hermitian_dense(heev_qr, n):
    """The complex Householder + QR solver of the block Lanczos matrices."""
    rng = np.random.default_rng(300 + n)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    check_heig(M + M.conj().T, *heev_qr(M + M.conj().T), rel=1e-13)


def test_complex_qr_graded_block_arrowhead(heev_qr):
    """The shape of a block thick-restart Lanczos matrix: kept Ritz values
    spanning many orders of magnitude, a block of complex couplings to them,
    then a block tridiagonal part with upper-triangular off-diagonal blocks."""
    n, k0, nb = 126, 42, 6
    rng = np.random.default_rng(11)
    A = np.zeros((n, n), dtype=np.complex128)
    A[np.arange(k0), np.arange(k0)] = 10.0 ** rng.uniform(0, 12, k0)
    C = (rng.standard_normal((nb, k0)) + 1j * rng.standard_normal((nb, k0))) * 1e-2
    A[k0:k0 + nb, :k0] = C
    A[:k0, k0:k0 + nb] = C.conj().T
    for j in range(k0, n, nb):
        D = rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))
        A[j:j + nb, j:j + nb] = 0.5 * (D + D.conj().T)
        if j + nb < n:
            R = np.triu(rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb)))
            A[j + nb:j + 2 * nb, j:j + nb] = R
            A[j:j + nb, j + nb:j + 2 * nb] = R.conj().T
    steps, w, Z = heev_qr(A)
    check_heig(A, steps, w, Z, rel=1e-13)
    ref = np.linalg.eigvalsh(A)
    big = ref > 1e3
    assert np.abs(w[big] - ref[big]).max() <= 1e-12 * ref[big].max()


def test_complex_qr_degenerate_and_real_input(heev_qr):
    """Exact degeneracies and a zero matrix; on a real symmetric matrix the
    complex solver gives the real solver's eigenvalues."""
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)))
    lam = np.repeat([0.5, 1.0, 3.0], 4)
    A = (Q * lam) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    check_heig(A, *heev_qr(A), rel=1e-13)
    steps, w, Z = heev_qr(np.zeros((3, 3)))
    assert np.all(w == 0)
    M = rng.standard_normal((30, 30))
    S = M + M.T
    steps, w, Z = heev_qr(S.astype(np.complex128))
    assert np.abs(w - np.linalg.eigvalsh(S)).max() <= 1e-13 * np.abs(S).max() * 30
