"""Closed forms that pin the oracle to the mathematics rather than to itself.

Free field (every link the identity, staggered phases and the antiperiodic
time sign folded in): the phases make the hopping terms of different
directions anticommute, so D^2 = sum_mu D_mu^2 with no phase left, a
translation-invariant operator.  On a plane wave of momentum p,
D_mu -> 2i (c1 sin p_mu + c3 sin 3 p_mu), hence

    -D^2 -> 4 sum_mu (c1 sin p_mu + c3 sin 3 p_mu)^2

with p_mu = 2 pi n / L_mu in space and p_t = pi (2n+1) / T in time.  The even
sites carry exactly half of every multiplicity (momenta p and p + (pi,...)
pair into one even and one odd combination), times 3 colours.
"""
from __future__ import annotations

import numpy as np


def momenta(dims):
    X, Y, Z, T = dims
    px = 2 * np.pi * np.arange(X) / X
    py = 2 * np.pi * np.arange(Y) / Y
    pz = 2 * np.pi * np.arange(Z) / Z
    pt = np.pi * (2 * np.arange(T) + 1) / T
    return px, py, pz, pt


def free_symbol(dims, c1, c3):
    """4 sum_mu (c1 sin p + c3 sin 3p)^2 on the grid [T][Z][Y][X] of momenta."""
    px, py, pz, pt = momenta(dims)
    PT, PZ, PY, PX = np.meshgrid(pt, pz, py, px, indexing="ij")
    f = lambda p: (c1 * np.sin(p) + c3 * np.sin(3 * p)) ** 2
    return 4 * (f(PX) + f(PY) + f(PZ) + f(PT))


def free_even_spectrum(dims, c1, c3, two_m=0.0):
    """Sorted eigenvalues of A = (2m)^2 - D_eo D_oe on even sites, free field."""
    full = np.sort(np.repeat(free_symbol(dims, c1, c3).ravel(), 3))
    return full[::2] + two_m * two_m


def free_solve_fft(dims, c1, c3, two_m, y):
    """Solve ((2m)^2 - D^2) psi = y on the full lattice by FFT (free field).

    psi(x) = exp(i pi t / T) phi(x) turns the antiperiodic problem into a
    periodic one whose time momenta are shifted by pi / T.
    """
    X, Y, Z, T = dims
    t = np.arange(T)[:, None, None, None, None]
    twist = np.exp(1j * np.pi * t / T)
    yp = y / twist
    yk = np.fft.fftn(yp, axes=(0, 1, 2, 3))
    kx = 2 * np.pi * np.fft.fftfreq(X)
    ky = 2 * np.pi * np.fft.fftfreq(Y)
    kz = 2 * np.pi * np.fft.fftfreq(Z)
    kt = 2 * np.pi * np.fft.fftfreq(T) + np.pi / T
    KT, KZ, KY, KX = np.meshgrid(kt, kz, ky, kx, indexing="ij")
    f = lambda p: (c1 * np.sin(p) + c3 * np.sin(3 * p)) ** 2
    sym = two_m * two_m + 4 * (f(KX) + f(KY) + f(KZ) + f(KT))
    phi = np.fft.ifftn(yk / sym[..., None], axes=(0, 1, 2, 3))
    return phi * twist
