"""Supports with additive structure on the GPU (Sec. IX-A, IX-B).

Lemma 5's algorithm: the Hi-DFT on all n pivots of a proper GAP (2^n samples,
one element per leaf node, mu* = 1), here Shift-and-Sample with r = every
pivot of J; and the cheaper Lemma-4 choice of r.  Expected values are seeded
coefficients whose samples the FP64 oracle synthesised; each recovery is held
to its plan's error bound (at most 1e-5 for every plan the library accepts).
"""
import numpy as np
import pytest

import oracle
from workloads import arithmetic_progression, complex_normal, gap_support, rng_for

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


def _sas_run(plan, f_rows):
    batch, n = f_rows.shape
    x = torch.from_numpy(f_rows.astype(np.complex64)).cuda()
    y = torch.full((batch, plan.k), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
    work = torch.empty(max(plan.workspace_bytes(batch) // 8, 1), dtype=torch.complex64,
                       device="cuda")
    plan.execute_ptr(x.data_ptr(), n, y.data_ptr(), plan.k, batch, work.data_ptr())
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.complex128)


def _check(M, J, plan, rng, tol):
    S = plan.samples().tolist()
    c = complex_normal((4, len(J)), rng)
    f = oracle.synthesize_samples(M, J, c, S)
    got = _sas_run(plan, f)
    err = oracle.rel_l2(got, c)
    print(f"  r={plan.pivots()} mu*={plan.mu_max} samples={plan.samples_per_signal} "
          f"rel-L2 max {np.max(err):.2e}", flush=True)
    assert tol <= 1e-5
    assert np.all(np.isfinite(got)) and np.max(err) <= tol


@pytest.mark.parametrize("sizes", [[64], [16, 16], [8, 8, 4], [32, 8], [4, 4, 4, 4],
                                   [128], [64, 4], [8, 16, 2]])
def test_gap_hidft_on_all_pivots(sizes):
    rng = rng_for(930, len(sizes) * 1000 + sizes[0])
    M = int(rng.integers(16, 25))
    g = gap_support(M, sizes, rng)
    J = g.J.tolist()
    P, _ = native.analyze(M, J)
    print(f"case GAP sizes={sizes} M={M} k={len(J)} pivots={len(P)}", flush=True)
    if len(P) > native.MAX_LOG2_K_LARGE:
        pytest.skip("more pivots than the executor's 2^22 samples")
    full = native.SASPlan(M, J, pivots=P)
    assert full.mu_max == 1
    _check(M, J, full, rng, full.err_bound)
    full.close()
    auto = native.SASPlan(M, J)
    assert oracle.is_part_homogeneous(M, J, auto.pivots())
    _check(M, J, auto, rng, auto.err_bound)
    auto.close()


@pytest.mark.parametrize("alpha", [0, 1, 5, 9])
def test_arithmetic_progressions(alpha):
    rng = rng_for(931, alpha)
    M = 20
    k = int(rng.integers(100, 1500))
    ap = arithmetic_progression(M, k, rng, alpha)
    J = ap.J.tolist()
    print(f"case AP alpha={alpha} k={k}", flush=True)
    auto = native.SASPlan(M, J)
    _check(M, J, auto, rng, auto.err_bound)
    auto.close()
    P, _ = native.analyze(M, J)
    full = native.SASPlan(M, J, pivots=P)
    assert full.mu_max == 1 and full.samples_per_signal == 1 << len(P)
    _check(M, J, full, rng, full.err_bound)
    full.close()


@pytest.mark.parametrize("kind,M,size,alpha", [("ap", 22, 20000, 1), ("ap", 22, 40000, 3),
                                              ("ap", 24, 100000, 5), ("gap", 24, [256, 64], 0),
                                              ("gap", 24, [64, 64, 16], 0),
                                              ("ap", 24, 1200000, 2), ("ap", 24, 3000000, 2)])
def test_more_pivots_than_one_signal_in_lds(kind, M, size, alpha):
    """Lemma 5's Hi-DFT on all n > 14 pivots (2^n samples, mu* = 1) runs in
    passes through a workspace; every coefficient against the seeded ones
    the samples were synthesised from (FP64, full-length inverse DFT), and
    hidft_sas_execute_noalloc gives the same bits.  n = 21 and 22 (the last
    two cases) take the three-group column pass and the subtree order that
    runs both signals of one subtree back to back, with the placement
    keeping 1.2 and 3 million of the 2^21 and 2^22 outputs."""
    rng = rng_for(932, M * 7 + (size if kind == "ap" else size[0]))
    J = (arithmetic_progression(M, size, rng, alpha) if kind == "ap"
         else gap_support(M, size, rng)).J.tolist()
    P, _ = native.analyze(M, J)
    print(f"case {kind} M={M} k={len(J)} pivots={len(P)}", flush=True)
    assert 14 < len(P) <= native.MAX_LOG2_K_LARGE
    plan = native.SASPlan(M, J, pivots=P)
    assert plan.mu_max == 1 and plan.samples_per_signal == 1 << len(P)
    assert plan.workspace_bytes(2) == 2 * (1 << len(P)) * 8
    S = plan.samples().tolist()
    c = complex_normal((2, len(J)), rng)
    f = oracle.synthesize_samples_fft(M, J, c, S)
    got = _sas_run(plan, f)
    err = oracle.rel_l2(got, c)
    print(f"  rel-L2 max {np.max(err):.2e} (bound {plan.err_bound:.2e})", flush=True)
    assert np.max(err) <= plan.err_bound <= 1e-5
    x = torch.from_numpy(f.astype(np.complex64)).cuda()
    y = torch.empty((2, plan.k), dtype=torch.complex64, device="cuda")
    if plan.workspace_bytes(1) <= native.SAS_SCRATCH_BYTES:
        plan.execute_noalloc_ptr(x.data_ptr(), len(S), y.data_ptr(), plan.k, 2)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().astype(np.complex128), got)
    else:  # one signal's workspace exceeds the static scratch: refused, nothing run
        with pytest.raises(native.HiDFTError, match="scratch"):
            plan.execute_noalloc_ptr(x.data_ptr(), len(S), y.data_ptr(), plan.k, 2)
    # the induced weights stay within one signal in LDS
    with pytest.raises(native.HiDFTError):
        native.SASPlan(M, J, pivots=P, weights_only=True)
    plan.close()
