"""GPU parity of the learned initial guess (an extension beyond the paper:
deflated CG stays the solver) against the FP64 oracle in
oracle/learned_guess.py: the network's output, the loss and its gradient, the
Adam update, BF16 inference, the fallback rule of hisq_nn_guess, and argument
errors.

Bars.  The library runs the network in FP32 (FP32 links, activations and
weights; FP64 sums for gradients and norms).  Three layers of nine FP32
transports accumulate a relative error of a few 1e-7 per output; the bars
below (1e-5 per sample for outputs and the loss, 1e-4 of the largest entry for
the gradient, whose entries are sums of ~10^5 products) leave a margin of ten
or more.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import hisq_oracle as O
from oracle import learned_guess as N
from paper_2502_00152_amd import inputs as I
from tests.gpu_util import Problem, dev, host, rel_per_rhs, to_parity

pytestmark = pytest.mark.gpu

RAGGED = (6, 6, 4, 6)  # 864 sites: three full blocks of 256 and a ragged tail


def params(seed):
    """Initial parameters with gates that depend on |psi| (a != 0)."""
    th = I.nn_initial_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    off = N.N_PARAMS - 4 * N.CH
    th[off:] = rng.uniform(-1.5, 1.5, size=4 * N.CH)
    return th.astype(np.float32)


def bf16(a):
    """Round float32 to bfloat16 (nearest, ties to even) and back."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def even_sources(dims, seeds):
    m = O.even_mask(dims)[..., None]
    return np.stack([I.gaussian_source(dims, s) * m for s in seeds])


@pytest.fixture(scope="module", params=[RAGGED, (8, 8, 8, 8)], ids=["ragged864", "8^4"])
def lat(request):
    pr = Problem(request.param, 0.5, 5101, 5102)
    pr.g = pr.gauge()
    pr.mask = O.even_mask(pr.dims)
    yield pr
    pr.g.close()


def oracle_apply(pr, th, r_full, normalize):
    out = []
    for r in r_full:
        s = np.linalg.norm(r) if normalize else 1.0
        out.append(N.apply(np.float64(th), pr.F, r / s, pr.mask) * s)
    return to_parity(np.stack(out), pr.dims, 0)


@pytest.mark.parametrize("flags", [0, 1], ids=["raw", "normalized"])
def test_forward_matches_oracle(lat, flags):
    import torch
    from paper_2502_00152_amd import hisq
    pr = lat
    th = params(11)
    r_full = even_sources(pr.dims, [21, 22, 23])
    ref = oracle_apply(pr, th, r_full, flags & 1)
    with hisq.Network(pr.g, th) as net:
        out = torch.zeros((3, 3, pr.g.vh), dtype=torch.complex128, device="cuda")
        hisq.hisq_nn_apply(net, dev(to_parity(r_full, pr.dims, 0)), out, flags)
        got = host(out)
    assert max(rel_per_rhs(got, ref)) < 1e-5


def test_bf16_inference_uses_rounded_weights(lat):
    import torch
    from paper_2502_00152_amd import hisq
    pr = lat
    th = params(12)
    r_full = even_sources(pr.dims, [31, 32])
    ref16 = oracle_apply(pr, bf16(th), r_full, True)
    ref32 = oracle_apply(pr, th, r_full, True)
    with hisq.Network(pr.g, th) as net:
        out = torch.zeros((2, 3, pr.g.vh), dtype=torch.complex128, device="cuda")
        hisq.hisq_nn_apply(net, dev(to_parity(r_full, pr.dims, 0)), out,
                           hisq.HISQ_NN_NORMALIZE | hisq.HISQ_NN_BF16)
        got = host(out)
        # the FP32 parameters are untouched by BF16 inference
        assert np.array_equal(hisq.hisq_nn_get_params(net), th)
    assert max(rel_per_rhs(got, ref16)) < 1e-5
    # and rounding the weights matters at this bar (the test can tell them apart)
    assert max(rel_per_rhs(ref16, ref32)) > 1e-4


@pytest.mark.parametrize("flags", [0, 1], ids=["raw", "normalized"])
def test_loss_and_gradient_match_oracle(lat, flags):
    from paper_2502_00152_amd import hisq
    pr = lat
    th = params(13)
    r_full = even_sources(pr.dims, [41, 42, 43])
    e_full = even_sources(pr.dims, [51, 52, 53])
    sc = [np.linalg.norm(r) if flags else 1.0 for r in r_full]
    L_ref, g_ref = N.loss_and_grad(np.float64(th), pr.F, [r / s for r, s in zip(r_full, sc)],
                                   [e / s for e, s in zip(e_full, sc)], pr.mask)
    with hisq.Network(pr.g, th) as net:
        L, g = hisq.hisq_nn_loss_grad(net, dev(to_parity(r_full, pr.dims, 0)),
                                      dev(to_parity(e_full, pr.dims, 0)), flags)
        # fixed-order sums: a second evaluation is bitwise identical
        L2, g2 = hisq.hisq_nn_loss_grad(net, dev(to_parity(r_full, pr.dims, 0)),
                                        dev(to_parity(e_full, pr.dims, 0)), flags)
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
    assert np.max(np.abs(g - g_ref)) <= 1e-4 * np.max(np.abs(g_ref))
    # every parameter block carries gradient (a dropped term shows here)
    for lo, hi in ((0, 72), (72, 648), (648, 720), (720, 736), (736, 752)):
        assert np.linalg.norm(g[lo:hi] - g_ref[lo:hi]) <= 1e-4 * np.linalg.norm(g_ref[lo:hi])
    assert L == L2 and np.array_equal(g, g2)


def test_adam_steps_match_oracle(lat):
    from paper_2502_00152_amd import hisq
    pr = lat
    th = params(14)
    r = dev(to_parity(even_sources(pr.dims, [61, 62]), pr.dims, 0))
    e = dev(to_parity(even_sources(pr.dims, [63, 64]), pr.dims, 0))
    lr = 3e-3
    with hisq.Network(pr.g, th) as net:
        with pytest.raises(hisq.HisqError):
            hisq.hisq_nn_adam_step(net, lr)  # no gradient yet
        ref = np.float64(th)
        m = np.zeros_like(ref)
        v = np.zeros_like(ref)
        for t in (1, 2, 3):
            _, g = hisq.hisq_nn_loss_grad(net, r, e)
            hisq.hisq_nn_adam_step(net, lr)
            ref, m, v = N.adam(ref, g, m, v, t, lr)
            got = hisq.hisq_nn_get_params(net)
            assert np.max(np.abs(got - ref)) <= 1e-6 * max(1.0, np.max(np.abs(ref)))
            assert np.max(np.abs(got - th)) > 0.5 * lr  # the step was taken


def test_train_lowers_the_loss(lat):
    from paper_2502_00152_amd import hisq
    pr = lat
    # targets e = r / 4: a network that learns the constant 1/4 fits them exactly
    r_full = even_sources(pr.dims, list(range(70, 78)))
    r = dev(to_parity(r_full, pr.dims, 0))
    e = dev(to_parity(r_full / 4.0, pr.dims, 0))
    with hisq.Network(pr.g, params(15)) as net:
        losses = hisq.hisq_nn_train(net, r, e, batch=4, steps=60, lr=1e-2)
        L_end, _ = hisq.hisq_nn_loss_grad(net, r, e)
        # the reported losses are those of the batches as trained
        net2 = hisq.Network(pr.g, params(15))
        L0, _ = hisq.hisq_nn_loss_grad(net2, r[:4].contiguous(), e[:4].contiguous())
        net2.close()
    assert abs(losses[0] - L0) <= 1e-12 * L0
    assert np.all(np.isfinite(losses))
    # the oracle, trained the same way in FP64, ends near 3e-4 of the first loss
    assert L_end < 1e-2 * losses[0]


def test_guess_keeps_only_improving_corrections(lat):
    import torch
    from paper_2502_00152_amd import hisq
    pr = lat
    two_m = 0.1
    b_full = even_sources(pr.dims, [81, 82])
    b = dev(to_parity(b_full, pr.dims, 0))
    x0 = to_parity(even_sources(pr.dims, [83, 84]), pr.dims, 0) * 0.1
    # N(r) = c r: identity transports on channel 0 only, constant gates s
    th = np.zeros(N.N_PARAMS, dtype=np.float32)
    th[0] = 1.0                      # W1[0][0][0]
    th[72] = 1.0                     # W2[0][0][0]
    off_g1, off_g2 = 720, 736
    th[off_g1 + 1] = 20.0            # b of gate 1, channel 0: s = 1 - 2e-9
    th[off_g2 + 1] = 20.0
    for c_lin, want in ((0.01, 1), (-0.01, 0)):
        th[648] = c_lin              # W3[0][0][0]
        with hisq.Network(pr.g, th) as net:
            x = dev(x0)
            kept = hisq.hisq_nn_guess(net, two_m, b, x)
            got = host(x)
        assert kept == [want, want]
        if want:
            # x + c s^2 r with r = b - A x0, A from the oracle
            r = b_full - np.stack([O.apply_A(pr.F, pr.L, two_m, xf)
                                   for xf in _full(x0, pr.dims)])
            s = 1.0 / (1.0 + np.exp(-20.0))
            ref = x0 + c_lin * s * s * to_parity(r, pr.dims, 0)
            assert max(rel_per_rhs(got, ref)) < 1e-6
        else:
            assert np.array_equal(got, x0)
    # a zero network never changes x
    with hisq.Network(pr.g) as net:
        x = dev(x0)
        assert hisq.hisq_nn_guess(net, two_m, b, x) == [0, 0]
        assert np.array_equal(host(x), x0)


def test_guess_projects_off_the_deflation_space():
    """With eigenpairs, x_new = x + d + V L^-1 V^H (r - A d), d = N(r): the
    composition written out with the oracle's network, A and Eq. (4); and the
    new residual has no component on the deflation space (Galerkin)."""
    import torch
    from paper_2502_00152_amd import hisq
    pr = Problem(RAGGED, 0.5, 5101, 5102)
    g = pr.gauge()
    dims, two_m, k = pr.dims, 0.05, 12
    mask = O.even_mask(dims)
    lam, Vc = O.lowest_eigenpairs(pr.F, pr.L, two_m, k, method="dense")
    evecs = np.concatenate([to_parity(O.from_compact(Vc[:, i], dims), dims, 0) for i in range(k)])
    eps = lam - two_m ** 2
    b_full = even_sources(dims, [91, 92])
    x0_full = np.stack([O.from_compact(O.deflation_guess(Vc, lam, O.to_compact(b, dims)), dims)
                        for b in b_full])
    th = params(17)
    try:
        for ev in (dev(evecs), dev(evecs.astype(np.complex64))):
            with hisq.Network(g, th) as net:
                x = dev(to_parity(x0_full, dims, 0))
                kept = hisq.hisq_nn_guess(net, two_m, dev(to_parity(b_full, dims, 0)), x,
                                          evecs=ev, evals=eps)
                got = host(x)
            for j in range(2):
                r = b_full[j] - O.apply_A(pr.F, pr.L, two_m, x0_full[j])
                s = np.linalg.norm(r)
                d = N.apply(np.float64(th), pr.F, r / s, mask) * s
                r1 = r - O.apply_A(pr.F, pr.L, two_m, d)
                c = O.from_compact(O.deflation_guess(Vc, lam, O.to_compact(r1, dims)), dims)
                x_ref = x0_full[j] + d + c
                r_new = b_full[j] - O.apply_A(pr.F, pr.L, two_m, x_ref)
                assert np.linalg.norm(Vc.conj().T @ O.to_compact(r_new, dims)) \
                    <= 1e-10 * np.linalg.norm(r)
                want = int(np.linalg.norm(r_new) < np.linalg.norm(r))
                assert kept[j] == want
                ref = to_parity(x_ref if want else x0_full[j], dims, 0)[0]
                # FP32 network and (second pass) FP32 eigenvectors: relative to |d|
                err = np.linalg.norm(got[j] - ref) / np.linalg.norm(to_parity(d, dims, 0))
                assert err < (1e-5 if ev.dtype == torch.complex128 else 1e-4)
    finally:
        g.close()


def _full(x_even, dims):
    from tests.gpu_util import from_parity
    return from_parity(x_even, dims, 0)


def test_argument_errors(lat):
    import torch
    from paper_2502_00152_amd import hisq
    pr = lat
    r = torch.zeros((2, 3, pr.g.vh), dtype=torch.complex128, device="cuda")
    e = torch.ones((2, 3, pr.g.vh), dtype=torch.complex128, device="cuda")
    L = hisq.lib()
    with hisq.Network(pr.g, params(16)) as net:
        for call in (
            lambda: hisq.hisq_nn_apply(net, r, r),                        # overlap
            lambda: hisq.hisq_nn_apply(net, r, e, flags=4),               # unknown flag
            lambda: hisq.hisq_nn_loss_grad(net, r, e, flags=hisq.HISQ_NN_BF16),
            lambda: hisq.hisq_nn_train(net, r, e, batch=3, steps=1, lr=1e-3),  # batch > pairs
            lambda: hisq.hisq_nn_guess(net, 0.0, e, r),                   # mass 0
        ):
            with pytest.raises(hisq.HisqError) as ei:
                call()
            assert ei.value.status == hisq.HISQ_ERR_INVALID_ARG
        # e = 0 makes the loss undefined
        with pytest.raises(hisq.HisqError) as ei:
            hisq.hisq_nn_loss_grad(net, e, r)
        assert ei.value.status == hisq.HISQ_ERR_NAN
        bad = np.full(N.N_PARAMS, np.nan, dtype=np.float32)
        with pytest.raises(hisq.HisqError):
            hisq.hisq_nn_set_params(net, bad)
        assert L.hisq_nn_apply(net.handle, r.data_ptr(), e.data_ptr(), 0, 0, None) == \
            hisq.HISQ_ERR_INVALID_ARG


def test_forward_48x48x48x96_sampled_sites():
    """The network at the size of one GPU's share of a large-lattice solve
    (48^3 x 96), in the launch configuration of inference, on sampled output
    sites.  N(r) at x depends on r and the links within three hops of x, so
    the oracle evaluates it on an 8^4 periodic window whose centre is x (index
    4 in each direction): wrapping corrupts one more layer of window sites per
    network layer, which after three layers leaves indices 3 and 4 exact.
    Centres have even coordinates (the window's staggered phases then equal
    the lattice's) and 4 <= t <= T - 4 (no antiperiodic time boundary inside
    the window), so folding the window's raw links reproduces the lattice's
    folded links there."""
    import torch
    from paper_2502_00152_amd import hisq
    dims = (48, 48, 48, 96)
    X, Y, Z, T = dims
    print(f"[48^3x96] drawing links", flush=True)
    W = I.random_su3_field_device(dims, 0.5, 48001)
    Nl = I.random_su3_field_device(dims, 0.5, 48002)
    g = hisq.Gauge(dims, W, Nl, I.C_FAT, I.C_LONG, 3)
    try:
        vh = g.vh
        gen = torch.Generator(device="cuda")
        gen.manual_seed(48003)
        r = torch.randn((1, 3, vh), dtype=torch.complex128, device="cuda", generator=gen)
        out = torch.zeros_like(r)
        th = params(18)
        with hisq.Network(g, th) as net:
            hisq.hisq_nn_apply(net, r, out, 0)
        torch.cuda.synchronize()
        print(f"[48^3x96] network applied", flush=True)
        rng = np.random.default_rng(48004)
        wdims = (8, 8, 8, 8)
        wmask = O.even_mask(wdims)
        off = np.arange(-4, 4)
        for _ in range(6):
            xc = [2 * int(rng.integers(0, L // 2)) for L in (X, Y, Z)]
            tc = 2 * int(rng.integers(2, T // 2 - 1))          # 4 <= tc <= T - 4
            cx = (xc[0] + off) % X
            cy = (xc[1] + off) % Y
            cz = (xc[2] + off) % Z
            ct = tc + off
            it, iz, iy, ix = np.meshgrid(ct, cz, cy, cx, indexing="ij")
            lex = ((it * Z + iz) * Y + iy) * X + ix              # [8][8][8][8]
            par = (ix + iy + iz + it) % 2
            li = torch.from_numpy(lex.reshape(-1)).cuda()
            Wwin = W.reshape(4, -1, 3, 3)[:, li].reshape(4, 8, 8, 8, 8, 3, 3).cpu().numpy()
            Nwin = Nl.reshape(4, -1, 3, 3)[:, li].reshape(4, 8, 8, 8, 8, 3, 3).cpu().numpy()
            Fw, _ = O.fold_links(Wwin, Nwin, I.C_FAT, I.C_LONG)
            cb = torch.from_numpy((lex.reshape(-1) >> 1)).cuda()
            rw = r[0][:, cb].T.reshape(8, 8, 8, 8, 3).cpu().numpy()
            rw = rw * (par == 0)[..., None]
            ref = N.apply(np.float64(th), Fw, rw, wmask)
            got = out[0][:, int(lex[4, 4, 4, 4]) >> 1].cpu().numpy()
            want = ref[4, 4, 4, 4]
            # scale: the typical output vector in the window's exact core
            scale = np.sqrt(np.mean(np.sum(np.abs(ref[3:5, 3:5, 3:5, 3:5]) ** 2, axis=-1)))
            assert np.linalg.norm(got - want) <= 1e-5 * max(np.linalg.norm(want), scale), \
                (xc, tc, got, want)
    finally:
        g.close()
        del W, Nl
        torch.cuda.empty_cache()
