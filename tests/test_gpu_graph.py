"""The grouped (uneven) launch and the fused launch inside a captured HIP graph.

Each is captured once on torch's capture stream and replayed several times,
with new samples copied in and other eager work and synchronisations between
the replays; every replay must equal the eager launch on the same data.
"""
import numpy as np
import pytest

from workloads import homogeneous_support, rng_for, sample_values

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2211_15299_amd.native")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _uneven(n, rng):
    plans, xs, ys = [], [], []
    for i in range(n):
        M = int(rng.integers(12, 25))
        s = int(rng.integers(6, min(14, M - 2) + 1))
        sup = homogeneous_support(M, s, rng)
        p = native.Plan(M, sup.J.tolist())
        plans.append(p)
        xs.append(torch.zeros(p.k, dtype=torch.complex64, device="cuda"))
        ys.append(torch.zeros(p.k, dtype=torch.complex64, device="cuda"))
    return plans, xs, ys


def test_grouped_launch_in_graph():
    rng = rng_for(3, 4242)
    plans, xs, ys = _uneven(96, rng)
    grp = native.Group([(p, x.data_ptr(), p.k, y.data_ptr(), p.k, 1)
                        for p, x, y in zip(plans, xs, ys)])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        grp.execute()          # warm-up outside capture (launch shape setup)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        grp.execute()
    for rep in range(3):
        data = [torch.from_numpy(sample_values(p.log2_n, p.k, 1, rng)[0]).cuda() for p in plans]
        for x, d in zip(xs, data):
            x.copy_(d)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [y.clone() for y in ys]
        _ = torch.randn(1 << 20, device="cuda").sum().item()   # other eager work
        grp.execute()
        torch.cuda.synchronize()
        for y, r in zip(ys, got):
            assert torch.equal(y, r), rep
    grp.close()


def test_fused_launch_in_graph():
    rng = rng_for(2, 4243)
    sup = homogeneous_support(20, 12, rng)
    plan = native.Plan(20, sup.J.tolist())
    x = torch.zeros((256, plan.k), dtype=torch.complex64, device="cuda")
    y = torch.zeros_like(x)
    plan.execute(x, out=y)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(x, out=y)
    for rep in range(3):
        x.copy_(torch.from_numpy(sample_values(20, plan.k, 256, rng)).cuda())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = y.clone()
        plan.execute(x, out=y)
        torch.cuda.synchronize()
        assert torch.equal(got, y), rep
