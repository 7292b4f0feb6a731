"""Oracle of the learned initial guess: a small gauge-covariant network that
maps the residual left by deflation to a correction of the solution.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/).  Plain PyTorch CPU ops in
float64; gradients by autograd.  This is an extension beyond the paper (which
solves with deflated CG only): the guess is x0 = x_defl + N(r0) with
r0 = b - A x_defl, and deflated CG stays the solver and decides what is kept.

Network N (8 channels, each channel a colour-vector field on the full lattice):
  layer(W, psi)^o = sum_d sum_c W[d, o, c] T_d psi^c
      T_0 = identity, T_{1+mu} psi(x) = F_mu(x) psi(x + mu),
      T_{5+mu} psi(x) = F_mu(x - mu)^H psi(x - mu)     (mu = x, y, z, t)
  with the folded fat links F (phases and boundary sign included) and real
  weights, so every layer commutes with gauge transformations;
  gate(a, b, psi)^c(x) = psi^c(x) sigmoid(a_c |psi^c(x)| + b_c)
      (a gauge-invariant scale per site and channel);
  N(r) = even part of layer(W3, gate(g2, layer(W2, gate(g1, layer(W1, r))))),
  W1 [9][8][1], W2 [9][8][8], W3 [9][1][8], g1, g2 [8][2] = (a_c, b_c).
Parameter vector order: W1, W2, W3, g1, g2, each C-order (752 numbers).
Loss of a batch: mean over samples of |N(r_s) - e_s|^2 / |e_s|^2.
"""
from __future__ import annotations

import numpy as np
import torch

CH = 8
SHAPES = (("W1", (9, CH, 1)), ("W2", (9, CH, CH)), ("W3", (9, 1, CH)),
          ("g1", (CH, 2)), ("g2", (CH, 2)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Split the flat parameter vector (torch) into named tensors."""
    out, k = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[k:k + n].reshape(shape)
        k += n
    return out


def transport(F, psi, d):
    """T_d psi for psi [C][T][Z][Y][X][3] (complex); F [4][T][Z][Y][X][3][3]."""
    if d == 0:
        return psi
    mu = (d - 1) % 4
    axis = 3 - mu          # lattice axis of direction mu in [T][Z][Y][X]
    if d <= 4:             # F_mu(x) psi(x + mu)
        nb = torch.roll(psi, -1, dims=1 + axis)
        return torch.einsum("tzyxab,ctzyxb->ctzyxa", F[mu], nb)
    Fb = torch.roll(F[mu], 1, dims=axis)   # F_mu(x - mu)
    nb = torch.roll(psi, 1, dims=1 + axis)
    return torch.einsum("tzyxba,ctzyxb->ctzyxa", Fb.conj(), nb)


def layer(F, W, psi):
    out = 0
    for d in range(9):
        out = out + torch.einsum("oc,ctzyxa->otzyxa", W[d].to(psi.dtype), transport(F, psi, d))
    return out


def gate(g, psi):
    n = torch.sqrt((psi.abs() ** 2).sum(-1))                # [C][T][Z][Y][X]
    s = torch.sigmoid(g[:, 0].reshape(-1, 1, 1, 1, 1) * n + g[:, 1].reshape(-1, 1, 1, 1, 1))
    return psi * s[..., None]


def network(theta, F, r, even_mask):
    """N(r) for one even-site input r [T][Z][Y][X][3]; returns the even part."""
    p = unpack(theta)
    a0 = r[None]
    a1 = gate(p["g1"], layer(F, p["W1"], a0))
    a2 = gate(p["g2"], layer(F, p["W2"], a1))
    z3 = layer(F, p["W3"], a2)[0]
    return z3 * even_mask[..., None]


def loss(theta, F, rs, es, even_mask):
    tot = 0
    for r, e in zip(rs, es):
        d = network(theta, F, r, even_mask) - e
        tot = tot + (d.abs() ** 2).sum() / (e.abs() ** 2).sum()
    return tot / len(rs)


def as_torch(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def loss_and_grad(theta_np, F_np, rs_np, es_np, even_mask_np):
    """Loss (float) and its gradient (numpy float64) at theta."""
    theta = torch.tensor(np.asarray(theta_np, dtype=np.float64), requires_grad=True)
    F = as_torch(F_np)
    rs = [as_torch(r) for r in rs_np]
    es = [as_torch(e) for e in es_np]
    m = as_torch(even_mask_np.astype(np.float64))
    L = loss(theta, F, rs, es, m)
    L.backward()
    return float(L.detach()), theta.grad.numpy().copy()


def apply(theta_np, F_np, r_np, even_mask_np):
    """N(r) as numpy."""
    with torch.no_grad():
        out = network(torch.tensor(np.asarray(theta_np, dtype=np.float64)), as_torch(F_np),
                      as_torch(r_np), as_torch(even_mask_np.astype(np.float64)))
    return out.numpy()


def adam(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba), t = step number starting at 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
