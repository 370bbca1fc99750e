"""Inverse transform (coefficients on J -> samples on I_r) against the oracle.

The oracle synthesises f_I = F^{-1}(I_r, J) c in FP64 (Sec. V-A); the GPU path
runs the adjoint of the radix-2 stages.  Also: inverse then forward recovers
c, and the two maps are adjoint up to N^2/k: the forward map is
(N/k) F(J, I_r) and the inverse (1/N) F(J, I_r)^H, so
<fwd g, c> = (N^2/k) <g, inv c>.
"""
import numpy as np
import pytest

import oracle
from workloads import complex_normal, homogeneous_support, rng_for

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


def _inverse(plan, c, ld_in=None, ld_out=None):
    batch, k = c.shape
    ld_in, ld_out = ld_in or k, ld_out or k
    x = torch.zeros((batch, ld_in), dtype=torch.complex64, device="cuda")
    x[:, :k] = torch.from_numpy(c.astype(np.complex64))
    y = torch.full((batch, ld_out), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
    plan.inverse_ptr(x.data_ptr(), ld_in, y.data_ptr(), ld_out, batch)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    assert np.all(np.isnan(out[:, k:]))
    return out[:, :k].astype(np.complex128)


@pytest.mark.parametrize("s", list(range(0, 15)))
def test_inverse_every_size_against_oracle(s):
    rng = rng_for(3000, s)
    M = int(rng.integers(max(s, 1), 25))
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    plan = native.Plan(M, J)
    batch = 5 if s < 12 else 2
    c = complex_normal((batch, len(J)), rng)
    got = _inverse(plan, c, ld_in=len(J) + 1, ld_out=len(J) + 2)
    I = plan.samples().tolist()
    if s <= 12:
        want = oracle.synthesize_samples(M, J, c, I)
        err = oracle.rel_l2(got, want)
    else:
        sel = rng.choice(len(I), 64, replace=False)
        want = oracle.synthesize_samples(M, J, c, [I[i] for i in sel])
        err = oracle.rel_l2(got[:, sel], want)
    assert np.max(err) <= 1e-5, (s, np.max(err))
    plan.close()


def test_round_trip_and_adjointness():
    rng = rng_for(3001, 0)
    for M, s in [(20, 12), (22, 14), (10, 6), (16, 9)]:
        sup = homogeneous_support(M, s, rng)
        plan = native.Plan(M, sup.J.tolist())
        k, N = plan.k, 1 << M
        c = complex_normal((4, k), rng)
        f = _inverse(plan, c)
        x = torch.from_numpy(f.astype(np.complex64)).cuda()
        back = plan.execute(x).cpu().numpy().astype(np.complex128)
        assert np.max(oracle.rel_l2(back, c)) <= 2e-5
        # <fwd g, c> = (N^2/k) <g, inv c> for random g, c
        g = complex_normal((1, k), rng) * np.sqrt(k) / N
        Fg = plan.execute(torch.from_numpy(g.astype(np.complex64)).cuda()).cpu().numpy()
        lhs = np.vdot(c[0], Fg[0].astype(np.complex128))
        rhs = (N * N / k) * np.vdot(f[0], g[0].astype(np.complex64).astype(np.complex128))
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs) + 1e-12
        plan.close()


def test_inverse_in_place_and_errors():
    rng = rng_for(3002, 0)
    sup = homogeneous_support(12, 8, rng)
    plan = native.Plan(12, sup.J.tolist())
    k = plan.k
    c = complex_normal((3, k), rng)
    want = _inverse(plan, c)
    x = torch.from_numpy(c.astype(np.complex64)).cuda()
    plan.inverse_ptr(x.data_ptr(), k, x.data_ptr(), k, 3)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy().astype(np.complex128), want)
    assert native.lib().hidft_execute_inverse(plan.handle, x.data_ptr(), k - 1, x.data_ptr(), k, 1,
                                              None) == 1
