"""hidft_sas_execute_noalloc: Shift-and-Sample without a workspace argument,
against hidft_sas_execute with one (bit for bit) and the oracle, on two calls
in a row, the second with a smaller batch."""
import numpy as np
import pytest

import oracle
from workloads import complex_normal, homogeneous_support, rng_for, sample_values

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2211_15299_amd.native")

SCRATCH = 16 << 20


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _half_of_homogeneous(seed, M, s, frac):
    rng = rng_for(960, seed)
    K = homogeneous_support(M, s, rng)
    keep = rng.random(len(K.J)) < frac
    return [int(j) for j, kp in zip(K.J, keep) if kp], rng


def _both(plan, x, batch):
    """(workspace path, allocation-free path) outputs of the first `batch` rows."""
    n = plan.samples_per_signal
    y_ws = torch.full((batch, plan.k), complex(np.nan, np.nan), dtype=torch.complex64,
                      device="cuda")
    y_na = torch.full_like(y_ws, complex(np.nan, np.nan))
    work = torch.empty(max(plan.workspace_bytes(batch) // 8, 1), dtype=torch.complex64,
                       device="cuda")
    plan.execute_ptr(x.data_ptr(), n, y_ws.data_ptr(), plan.k, batch, work.data_ptr())
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    plan.execute_noalloc_ptr(x.data_ptr(), n, y_na.data_ptr(), plan.k, batch)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, "the allocation-free call changed the device's free memory"
    return y_ws, y_na


CASES = {
    # (M, s, kept fraction, seed, pivots left out of r)
    # a random half, r = all pivots but the top one: mu* = 2, about 24 KB of
    # shifted outputs per signal (681 signals per chunk)
    "half_mu2": (20, 12, 0.5, 0, 1),
    # a 90 % subset, r = all but three pivots: mu* = 8 (the solve's loop over
    # mu(v)), 16 KB per signal
    "subset_mu8": (14, 11, 0.9, 0, 3),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_noalloc_matches_workspace_path_on_two_calls(name):
    M, s, frac, seed, drop = CASES[name]
    J, rng = _half_of_homogeneous(seed, M, s, frac)
    P, _ = native.analyze(M, J)
    plan = native.SASPlan(M, J, pivots=P[: len(P) - drop], two_pass=True)
    assert plan.mu_max > 1 and plan.workspace_bytes(1) > 0
    per_signal = plan.mu_max * plan.n_nodes * 8
    print(f"case {name}: k={plan.k} mu*={plan.mu_max} nodes={plan.n_nodes} "
          f"{per_signal} B per signal, {SCRATCH // per_signal} signals per chunk", flush=True)
    n = plan.samples_per_signal
    first = max(3 * (SCRATCH // per_signal) - 7, 50)     # several chunks, a ragged last one
    x = torch.from_numpy(sample_values(M, n, first, rng)).cuda()
    # call 1: the large batch
    y_ws, y_na = _both(plan, x, first)
    assert torch.equal(y_ws.view(torch.float32), y_na.view(torch.float32))
    # call 2: a smaller batch of seeded signals, also against the oracle
    c = complex_normal((37, plan.k), rng)
    f = oracle.synthesize_samples_fft(M, J, c, plan.samples().tolist())
    x2 = torch.from_numpy(f.astype(np.complex64)).cuda()
    y_ws2, y_na2 = _both(plan, x2, 37)
    assert torch.equal(y_ws2.view(torch.float32), y_na2.view(torch.float32))
    err = oracle.rel_l2(y_na2.cpu().numpy().astype(np.complex128), c)
    print(f"  second call: rel-L2 max {np.max(err):.2e} (bound {plan.err_bound:.2e})", flush=True)
    assert np.max(err) <= plan.err_bound <= 1e-5
    plan.close()


def test_noalloc_without_workspace_paths():
    """Plans that need no workspace (mu* = 1, the one-kernel form) run as in
    hidft_sas_execute, bit for bit, on two calls in a row."""
    J, rng = _half_of_homogeneous(0, 20, 12, 0.5)
    P, _ = native.analyze(20, J)
    for plan in (native.SASPlan(20, J), native.SASPlan(20, J, pivots=P)):
        assert plan.workspace_bytes(100) == 0
        n = plan.samples_per_signal
        x = torch.from_numpy(sample_values(20, n, 300, rng)).cuda()
        for batch in (300, 11):
            y_ws, y_na = _both(plan, x, batch)
            assert torch.equal(y_ws.view(torch.float32), y_na.view(torch.float32))
        plan.close()


def test_noalloc_errors():
    J, rng = _half_of_homogeneous(0, 20, 12, 0.5)
    plan = native.SASPlan(20, J, two_pass=True)
    n = plan.samples_per_signal
    x = torch.zeros((2, n), dtype=torch.complex64, device="cuda")
    y = torch.zeros((2, plan.k), dtype=torch.complex64, device="cuda")
    with pytest.raises(native.HiDFTError):          # leading dimension below a row
        plan.execute_noalloc_ptr(x.data_ptr(), n - 1, y.data_ptr(), plan.k, 2)
    with pytest.raises(native.HiDFTError):          # output overlapping the input
        plan.execute_noalloc_ptr(x.data_ptr(), n, x.data_ptr(), plan.k, 2)
    plan.execute_noalloc_ptr(x.data_ptr(), n, y.data_ptr(), plan.k, 0)   # batch 0: no-op
    w = native.SASPlan(20, J, pivots=plan.pivots(), weights_only=True)
    with pytest.raises(native.HiDFTError) as ei:
        w.execute_noalloc_ptr(x.data_ptr(), n, y.data_ptr(), plan.k, 2)
    assert ei.value.status_name == "HIDFT_ERR_UNSUPPORTED"
    plan.close()
    w.close()
