"""GPU parity of the uneven batch at its full sizes: 8^4 (32 RHS), 12^4 (16),
16^3 x 32 (8) and 24^3 x 48 (4), each at 2m = 0.1, 0.02 and 0.005, eps 0.3
(batching of uneven solves, the paper's future work in section 4).  Each
lattice is one system with its three masses in one batched solve (a mass per
RHS, shared link loads); the four systems run concurrently.

Links are drawn on the device and copied to the host for the oracle (the
host draw of 24^3 x 48 takes about a minute).  Checks: every RHS converges;
the oracle's FP64 true residual of every RHS meets tol, and the library's
reported true residual of every RHS agrees with the oracle's (5% plus the
rounding of b - A x); the concurrent batched solve equals separate
single-mass solves bitwise for the smallest lattice; launching every chunk
of iterations of the four systems as one captured graph gives bitwise the
same solutions and iteration counts as one stream per system.
"""
from __future__ import annotations

import time

import numpy as np
import pytest

from oracle import hisq_oracle as O
from paper_2502_00152_amd import inputs as I
from tests.gpu_util import from_parity, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    import torch
    from paper_2502_00152_amd import hisq
    B = I.UNEVEN_BATCH
    t0 = time.time()
    lat = []
    for l, (dims, nrhs) in enumerate(B["lattices"]):
        Wd = I.random_su3_field_device(dims, B["eps"], 30000 + 1000 * l + 1)
        Nd = I.random_su3_field_device(dims, B["eps"], 30000 + 1000 * l + 2)
        g = hisq.Gauge(dims, Wd, Nd, I.C_FAT, I.C_LONG)
        F, L = O.fold_links(Wd.cpu().numpy(), Nd.cpu().numpy(), I.C_FAT, I.C_LONG)
        del Wd, Nd
        bs = []
        for k in range(len(B["masses"])):
            gen = torch.Generator(device="cuda")
            gen.manual_seed(30000 + 1000 * l + 100 + 10 * k)
            bs.append(torch.randn((nrhs, 3, g.vh), dtype=torch.complex128, device="cuda",
                                  generator=gen))
        lat.append(dict(dims=dims, nrhs=nrhs, g=g, F=F, L=L, b=torch.cat(bs),
                        masses=np.repeat(B["masses"], nrhs)))
    torch.cuda.empty_cache()
    print(f"[uneven] setup {time.time() - t0:.0f}s", flush=True)
    yield lat
    for d in lat:
        d["g"].close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "half"])
def test_uneven_batch_concurrent(batch, prec):
    import torch
    from paper_2502_00152_amd import hisq
    sp = {"fp64": hisq.HISQ_FP64, "fp32": hisq.HISQ_FP32, "half": hisq.HISQ_HALF}[prec]
    systems = [(d["g"], d["masses"], d["b"], torch.zeros_like(d["b"])) for d in batch]
    t0 = time.time()
    res = hisq.hisq_cg_solve_multi(systems, tol=1e-10, sloppy_prec=sp)
    torch.cuda.synchronize()
    n = sum(d["b"].shape[0] for d in batch)
    print(f"[uneven] {prec}: {n} solves in {time.time() - t0:.2f}s, iterations "
          f"{[max(r.iterations) for r in res]}", flush=True)
    worst = 0.0
    for d, (g, ms, b, x), r in zip(batch, systems, res):
        assert all(r.converged)
        xs, bs = host(x), host(b)
        for j in range(bs.shape[0]):
            xe = from_parity(xs[j:j + 1], d["dims"], 0)[0]
            be = from_parity(bs[j:j + 1], d["dims"], 0)[0]
            tr = O.norm(be - O.apply_A(d["F"], d["L"], ms[j], xe)) / O.norm(be)
            assert tr <= 1e-10, (d["dims"], j, ms[j], tr)
            # rounding of b - A x: terms of size lambda_max ||x||, lambda_max
            # <= (2m)^2 + 69.4 for unitary links
            slack = 64 * 2.0 ** -53 * (ms[j] ** 2 + 69.4) * O.norm(xe) / O.norm(be)
            gap = abs(r.true_residual[j] - tr)
            assert gap <= 0.05 * tr + slack, (d["dims"], j, ms[j], r.true_residual[j], tr)
            worst = max(worst, tr)
    print(f"[uneven] {prec}: largest oracle true residual {worst:.3e}", flush=True)
    # the smallest lattice: equal to separate single-mass solves
    d = batch[0]
    x = systems[0][3]
    nr = d["nrhs"]
    for k, m in enumerate(I.UNEVEN_BATCH["masses"]):
        xk = torch.zeros_like(d["b"][k * nr:(k + 1) * nr])
        rk = hisq.hisq_cg_solve(d["g"], m, d["b"][k * nr:(k + 1) * nr].clone(), xk, tol=1e-10,
                                sloppy_prec=sp)
        assert rk.iterations == res[0].iterations[k * nr:(k + 1) * nr]
        assert torch.equal(xk, x[k * nr:(k + 1) * nr])


@pytest.mark.parametrize("prec", ["fp64", "half"])
def test_uneven_batch_one_graph_per_chunk(batch, prec):
    import torch
    from paper_2502_00152_amd import hisq
    sp = {"fp64": hisq.HISQ_FP64, "half": hisq.HISQ_HALF}[prec]
    out = {}
    try:
        for mode in (0, 1):
            hisq.hisq_set_tuning("cg_multi_graph", mode)
            systems = [(d["g"], d["masses"], d["b"], torch.zeros_like(d["b"])) for d in batch]
            t0 = time.time()
            res = hisq.hisq_cg_solve_multi(systems, tol=1e-10, sloppy_prec=sp)
            torch.cuda.synchronize()
            out[mode] = (res, [x for (_, _, _, x) in systems], time.time() - t0)
    finally:
        hisq.hisq_set_tuning("cg_multi_graph", -1)
    print(f"[uneven] {prec}: streams {out[0][2]:.3f}s, one graph per chunk {out[1][2]:.3f}s",
          flush=True)
    for r0, r1, x0, x1 in zip(out[0][0], out[1][0], out[0][1], out[1][1]):
        assert all(r1.converged)
        assert r0.iterations == r1.iterations
        assert torch.equal(x0, x1)
