"""Pins of the learned-guess oracle (oracle/learned_guess.py) against facts
that do not come from the oracle itself: gauge covariance, linearity when the
gates are constant, the identity network, a brute-force site loop for the
transports, adjointness of the forward and backward hops, finite-difference
gradients and the first Adam step."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import hisq_oracle as O
from oracle import learned_guess as N
from paper_2502_00152_amd import inputs as I

DIMS = (4, 4, 4, 6)


def links(dims=DIMS, seed=3):
    W = I.random_su3_field(dims, 0.5, seed)
    Lg = I.random_su3_field(dims, 0.5, seed + 1)
    return O.fold_links(W, Lg, I.C_FAT, I.C_LONG)[0]


def even_input(dims, seed):
    r = I.gaussian_source(dims, seed)
    return r * O.even_mask(dims)[..., None]


def test_transport_matches_site_loop():
    F = links()
    psi = I.gaussian_source(DIMS, 5)[None]
    X, Y, Z, T = DIMS
    rng = np.random.default_rng(0)
    for d in range(1, 9):
        got = N.transport(torch.from_numpy(F), torch.from_numpy(psi), d).numpy()[0]
        mu = (d - 1) % 4
        for _ in range(6):
            c = [int(rng.integers(0, n)) for n in DIMS]
            idx = lambda q: (q[3], q[2], q[1], q[0])
            if d <= 4:
                n = list(c); n[mu] = (c[mu] + 1) % DIMS[mu]
                ref = F[mu][idx(c)] @ psi[0][idx(n)]
            else:
                n = list(c); n[mu] = (c[mu] - 1) % DIMS[mu]
                ref = F[mu][idx(n)].conj().T @ psi[0][idx(n)]
            assert np.allclose(got[idx(c)], ref, rtol=1e-14, atol=1e-14)


def test_forward_and_backward_hops_are_adjoint():
    F = torch.from_numpy(links())
    a = torch.from_numpy(I.gaussian_source(DIMS, 6)[None])
    b = torch.from_numpy(I.gaussian_source(DIMS, 7)[None])
    for mu in range(4):
        lhs = torch.vdot(b.ravel(), N.transport(F, a, 1 + mu).ravel())
        rhs = torch.vdot(N.transport(F, b, 5 + mu).ravel(), a.ravel())
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gauge_covariance():
    F = links()
    Om = I.random_gauge_transform(DIMS, 11)
    Fp = np.empty_like(F)
    for mu in range(4):
        Fp[mu] = Om @ F[mu] @ np.roll(Om, -1, axis=3 - mu).conj().swapaxes(-1, -2)
    theta = I.nn_initial_params(1).astype(np.float64)
    theta[-32:] = np.tile([0.7, 0.3], 16)   # gates with a != 0 (nonlinear)
    m = O.even_mask(DIMS)
    r = even_input(DIMS, 12)
    rp = np.einsum("...ab,...b->...a", Om, r)
    lhs = N.apply(theta, Fp, rp, m)
    rhs = np.einsum("...ab,...b->...a", Om, N.apply(theta, F, r, m))
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_linear_when_gates_are_constant():
    F = links()
    theta = I.nn_initial_params(2).astype(np.float64)   # a = 0: gates are constants
    m = O.even_mask(DIMS)
    r1, r2 = even_input(DIMS, 13), even_input(DIMS, 14)
    al = 0.3 - 1.7j
    lhs = N.apply(theta, F, al * r1 + r2, m)
    rhs = al * N.apply(theta, F, r1, m) + N.apply(theta, F, r2, m)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_identity_network():
    F = links()
    theta = np.zeros(N.N_PARAMS)
    p = N.unpack(torch.from_numpy(theta))
    p["W1"][0, 0, 0] = 1.0
    p["W2"][0, 0, 0] = 1.0
    p["W3"][0, 0, 0] = 1.0
    p["g1"][:, 1] = 60.0   # sigmoid(60) = 1 to double precision
    p["g2"][:, 1] = 60.0
    m = O.even_mask(DIMS)
    r = even_input(DIMS, 15)
    assert np.abs(N.apply(theta, F, r, m) - r).max() <= 1e-15 * np.abs(r).max() + 1e-300


def test_gradient_matches_finite_differences():
    F = links()
    m = O.even_mask(DIMS)
    theta = I.nn_initial_params(3).astype(np.float64)
    theta[-32:] = np.tile([0.5, 0.2], 16)
    rs = [even_input(DIMS, 20 + j) for j in range(2)]
    es = [even_input(DIMS, 30 + j) for j in range(2)]
    L0, g = N.loss_and_grad(theta, F, rs, es, m)
    rng = np.random.default_rng(4)
    for k in list(rng.choice(N.N_PARAMS, 12, replace=False)) + [N.N_PARAMS - 1, N.N_PARAMS - 18]:
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (N.loss_and_grad(tp, F, rs, es, m)[0] - N.loss_and_grad(tm, F, rs, es, m)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k


def test_first_adam_step_is_signed_learning_rate():
    g = np.array([3.0, -1e-3, 0.0, 2e-9])
    th, m, v = N.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(th[:2], [-0.01, 0.01], rtol=1e-4)
    assert th[2] == 0.0
    assert abs(th[3]) < 0.01   # |g| comparable to eps: a damped step


def test_gates_hand_computed_at_one_site():
    """A hand-worked value with non-zero gate slopes a.  The weights keep only
    the identity hop and channel 0, and the input is zero except at one site
    where r = (3+4i, 12i, 0), so |r| = sqrt(9 + 16 + 144) = 13 (the norm of the
    colour vector, not of a single colour, not squared):
      gate 1, a = 0.1, b = -1.3:  sigmoid(0.1 * 13 - 1.3) = sigmoid(0) = 1/2,
          z = (1.5+2i, 6i, 0), |z| = sqrt(2.25 + 4 + 36) = 6.5;
      gate 2, a = 0.2, b = -0.3:  sigmoid(0.2 * 6.5 - 0.3) = sigmoid(1) = e/(1+e)
          = 0.7310585786300049,
      N(r) = z e/(1+e) = (1.0965878679450074 + 1.4621171572600098i,
                          4.3863514717800295i, 0) at that site, 0 elsewhere.
    A gate on |r|^2, on each colour separately, or with the sign of a or b
    flipped gives another value."""
    dims = (4, 4, 4, 4)
    F = links(dims)
    p = {k: np.zeros(s) for k, s in N.SHAPES}
    p["W1"][0, 0, 0] = 1.0
    p["W2"][0, 0, 0] = 1.0
    p["W3"][0, 0, 0] = 1.0
    p["g1"][0] = (0.1, -1.3)
    p["g2"][0] = (0.2, -0.3)
    theta = np.concatenate([p[k].ravel() for k, _ in N.SHAPES])
    r = np.zeros((4, 4, 4, 4, 3), dtype=np.complex128)
    site = (2, 1, 3, 0)  # [t][z][y][x], an even site
    assert sum(site) % 2 == 0
    r[site] = (3 + 4j, 12j, 0)
    out = N.apply(theta, F, r, O.even_mask(dims))
    want = np.array([1.0965878679450074 + 1.4621171572600098j, 4.3863514717800295j, 0])
    assert np.allclose(out[site], want, rtol=1e-15, atol=1e-15)
    out[site] = 0
    assert np.abs(out).max() == 0.0
