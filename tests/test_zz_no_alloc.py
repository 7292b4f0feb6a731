"""hisq_mdagm_noalloc (the allocation-free variant of hisq_mdagm) against
hisq_mdagm through the C ABI: the same kernels and launch shapes, so the
results must be equal bit for bit; two calls in a row with the second on a
smaller input, FP64 and FP32, two handles; no device memory taken by the call;
a request larger than the fixed scratch rejected before any launch; and the
call recorded in a HIP graph, replayed with eager work in between."""
from __future__ import annotations

import pytest

from paper_2502_00152_amd import inputs as I
from tests.gpu_util import Problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handles():
    big = Problem((16, 16, 16, 32), 0.5, 7101, 7102)
    small = Problem((8, 8, 8, 8), 0.3, 7201, 7202)
    big.g, small.g = big.gauge(), small.gauge()
    yield big, small
    big.g.close()
    small.g.close()


def rand(vh, nrhs, dtype, seed):
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    return torch.randn((nrhs, 3, vh), dtype=dtype, device="cuda", generator=gen)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_mdagm_twice_second_smaller(handles, prec):
    import torch
    from paper_2502_00152_amd import hisq
    big, small = handles
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    p = hisq.HISQ_FP64 if prec == "fp64" else hisq.HISQ_FP32
    # (handle, nrhs, 2m): the second call of each pair is smaller
    calls = [(big, 12 if prec == "fp64" else 24, 0.01), (big, 3, 0.05),
             (small, 40, 0.1), (small, 1, 0.2)]
    if prec == "fp32":  # the FP32 links exist after one allocating call
        for pr in (big, small):
            x = rand(pr.g.vh, 1, dt, 1)
            hisq.hisq_mdagm(pr.g, 0.1, x, torch.empty_like(x), prec=p)
    for k, (pr, nrhs, two_m) in enumerate(calls):
        x = rand(pr.g.vh, nrhs, dt, 100 + k)
        want = torch.empty_like(x)
        got = torch.full_like(x, float("nan"))
        hisq.hisq_mdagm(pr.g, two_m, x, want, prec=p)
        hisq.hisq_mdagm_noalloc(pr.g, two_m, x, got, prec=p)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (prec, k)


def test_noalloc_takes_no_device_memory_and_rejects_oversize(handles):
    import torch
    from paper_2502_00152_amd import hisq
    big, _ = handles
    # a fresh handle: hisq_mdagm would grow its scratch, the no-alloc call must not
    pr = Problem((12, 12, 12, 12), 0.4, 7301, 7302)
    g = pr.gauge()
    try:
        x = rand(g.vh, 8, torch.complex128, 5)
        y = torch.empty_like(x)
        hisq.hisq_mdagm_noalloc(g, 0.05, x, y)  # first call: symbol lookup
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for _ in range(3):
            hisq.hisq_mdagm_noalloc(g, 0.05, x, y)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        ref = torch.empty_like(x)
        hisq.hisq_mdagm(g, 0.05, x, ref)
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
    finally:
        g.close()
    # 16^3 x 32 with 24 FP64 RHS needs 3 * 65536 * 24 * 16 B = 75.5 MB > 64 MiB
    x = rand(big.g.vh, 24, torch.complex128, 6)
    y = torch.zeros_like(x)
    with pytest.raises(hisq.HisqError) as e:
        hisq.hisq_mdagm_noalloc(big.g, 0.01, x, y)
    assert e.value.status == hisq.HISQ_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.count_nonzero(y) == 0
    assert 3 * big.g.vh * 24 * 16 > hisq.NOALLOC_SCRATCH_BYTES


def test_noalloc_in_a_captured_graph(handles):
    """Recorded once into a HIP graph, replayed three times with eager work
    and synchronisations in between; every replay equals the eager result."""
    import torch
    from paper_2502_00152_amd import hisq
    _, small = handles
    two_m = 0.1
    x = rand(small.g.vh, 6, torch.complex128, 9)
    y = torch.empty_like(x)
    ref = torch.empty_like(x)
    hisq.hisq_mdagm(small.g, two_m, x, ref)
    hisq.hisq_mdagm_noalloc(small.g, two_m, x, y)  # warm: symbol lookup outside capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            hisq.hisq_mdagm_noalloc(small.g, two_m, x, y)
    torch.cuda.current_stream().wait_stream(s)
    for k in range(3):
        y.fill_(float("nan"))
        other = rand(small.g.vh, 6, torch.complex128, 50 + k)
        hisq.hisq_mdagm(small.g, 0.3, other, torch.empty_like(other))  # eager work between
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), k
    del graph
