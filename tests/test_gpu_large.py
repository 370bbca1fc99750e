"""GPU parity of transforms with more than 2^14 points.

Above one signal per LDS the plan splits the recursion (Corollary 2): the
top stages run per column, the rest per subtree, and a gather puts the
coefficients in the caller's order (three kernels through a workspace).
Checks, through the C ABI:
  * every coefficient of seeded transforms (k = 2^15..2^22) against the
    coefficients the samples were synthesised from (FP64 full-length inverse
    DFT read at I_r), and seeded positions of the same rows against the FP64
    oracle;
  * batches (k = 2^15, 2^19, 2^20): every row on up to 64 seeded positions
    of its own against the oracle and on the energy identity
    ||c||^2 = (N^2/k) ||f_I||^2 (Lemma 1);
  * hidft_execute (stream-ordered workspace), hidft_execute_ws (caller's
    workspace), in place, strided rows and a captured graph give the same
    bits;
  * the split twiddle table holds every twiddle rounded once from FP64;
  * the inverse map (the adjoint passes in reverse) against the samples the
    FP64 oracle synthesises from seeded coefficients, and forward after
    inverse returns the coefficients;
  * the calls that need one signal in LDS refuse these plans.
"""
import sys

import numpy as np
import pytest

import oracle
from tests.positions import positions_vs_oracle
from workloads import complex_normal, homogeneous_support, rng_for, sample_values

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2211_15299_amd.native")

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _energy_rel(c, f, M, k):
    N = float(1 << M)
    e_c = np.sum(np.abs(c.astype(np.complex128)) ** 2, axis=-1)
    e_f = (N * N / k) * np.sum(np.abs(f.astype(np.complex128)) ** 2, axis=-1)
    return np.abs(e_c - e_f) / e_f


@pytest.mark.parametrize("M,s", [(20, 15), (22, 16), (24, 17), (24, 18), (24, 19), (24, 20),
                                 (24, 21), (24, 22)])
def test_large_recovers_every_coefficient(M, s):
    rng = rng_for(4100, s)
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    plan = native.Plan(M, J)
    k = plan.k
    assert k == 1 << s and plan.workspace_bytes(2) == 2 * k * 8
    I = plan.samples().tolist()
    c = complex_normal((2, k), rng)
    f = oracle.synthesize_samples_fft(M, J, c, I).astype(np.complex64)
    _say(f"large: M={M} s={s} k={k}, 2 rows")
    x = torch.from_numpy(f).cuda()
    got = plan.execute(x).cpu().numpy()
    err = oracle.rel_l2(got.astype(np.complex128), c)
    _say(f"large: every coefficient against the synthesised ones, rel-L2 {np.max(err):.3e}")
    assert np.max(err) <= TOL, err
    n_pos = min(256, (1 << 25) // k)  # the oracle's submatrix stays within 512 MB
    pe = positions_vs_oracle(M, J, I, f, got, n_pos, rng_for(4101, s))
    _say(f"large: {n_pos} positions per row against the oracle, rel-L2 {np.max(pe):.3e}")
    assert np.max(pe) <= TOL, pe
    plan.close()


@pytest.mark.parametrize("M,s,batch", [(18, 15, 96), (22, 19, 6), (22, 20, 3), (22, 21, 3),
                                         (22, 21, 1)])
def test_large_batch_every_row(M, s, batch):
    """Chunks of 4096 outputs (s = 15) and of 16384 (s = 19..21: s1 = 7..9),
    the column pass in registers (s1 = 3), in two groups (s1 = 7, 8) and in
    three (s1 = 9), where the subtree pass runs the batch's signals of one
    subtree back to back (three signals: not a power of two; one signal:
    the signal-major order)."""
    rng = rng_for(4102, s)
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    plan = native.Plan(M, J)
    k = plan.k
    I = plan.samples().tolist()
    f = sample_values(M, k, batch, rng)
    x = torch.from_numpy(f).cuda()
    y = plan.execute(x)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    n_pos = min(64, (1 << 25) // k)  # the oracle's submatrix stays within 512 MB
    pe = positions_vs_oracle(M, J, I, f, got, n_pos, rng_for(4103, s), group=16)
    _say(f"large batch: s={s}, {batch} rows on {n_pos} positions each, "
         f"rel-L2 max {np.max(pe):.3e}")
    assert np.max(pe) <= TOL
    en = _energy_rel(got, f, M, k)
    assert np.max(en) <= 2 * TOL, np.max(en)
    # hidft_execute (stream-ordered workspace) gives the same bits
    z = torch.full_like(x, complex(np.nan, np.nan))
    plan.execute_ptr(x.data_ptr(), k, z.data_ptr(), k, batch)
    torch.cuda.synchronize()
    assert torch.equal(z, y)
    # strided rows through the caller's workspace
    xs = torch.zeros((batch, k + 5), dtype=torch.complex64, device="cuda")
    xs[:, :k] = x
    ys = torch.full((batch, k + 3), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
    wb = plan.workspace_bytes(batch)
    work = torch.empty(wb // 8, dtype=torch.complex64, device="cuda")
    plan.execute_ws_ptr(xs.data_ptr(), k + 5, ys.data_ptr(), k + 3, batch, work.data_ptr(), wb)
    torch.cuda.synchronize()
    assert torch.equal(ys[:, :k], y)
    assert torch.isnan(ys[:, k:]).all()  # nothing written past k
    # in place
    w = x.clone()
    plan.execute_ws_ptr(w.data_ptr(), k, w.data_ptr(), k, batch, work.data_ptr(), wb)
    torch.cuda.synchronize()
    assert torch.equal(w, y)
    plan.close()


@pytest.mark.parametrize("M,s,batch", [(19, 16, 8), (22, 21, 2)])
def test_large_in_a_graph(M, s, batch):
    """The caller-workspace forward and inverse passes captured in HIP graphs
    (s = 16: the column pass in registers; s = 21: the three-group column
    kernels and the subtree order of s1 = 9): every replay, with eager work
    in between, equals the eager launch."""
    rng = rng_for(4104, s)
    plan = native.Plan(M, homogeneous_support(M, s, rng).J.tolist())
    k = plan.k
    x = torch.from_numpy(sample_values(M, k, batch, rng)).cuda()
    ref = plan.execute(x)
    ref_inv = torch.empty_like(x)
    plan.inverse_ptr(ref.data_ptr(), k, ref_inv.data_ptr(), k, batch)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    wb = plan.workspace_bytes(batch)
    work = torch.empty(wb // 8, dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute_ws_ptr(x.data_ptr(), k, y.data_ptr(), k, batch, work.data_ptr(), wb,
                            stream=torch.cuda.current_stream())
    gi = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gi):
        plan.inverse_ws_ptr(ref.data_ptr(), k, z.data_ptr(), k, batch, work.data_ptr(), wb,
                            stream=torch.cuda.current_stream())
    for rep in range(3):
        y.fill_(complex(np.nan, np.nan))
        z.fill_(complex(np.nan, np.nan))
        work.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), f"forward replay {rep}"
        gi.replay()
        torch.cuda.synchronize()
        assert torch.equal(z, ref_inv), f"inverse replay {rep}"
    plan.close()


def test_large_twiddles_are_fp64_rounded_once():
    rng = rng_for(4105, 0)
    for M, s in [(20, 16), (40, 18), (30, 21)]:
        plan = native.Plan(M, homogeneous_support(M, s, rng).J.tolist())
        fp, num, den = plan.schedule()
        tw = plan.twiddles()
        exact = np.exp(-1j * np.pi * (num.astype(np.float64) / np.exp2(den.astype(np.float64))))
        for part_gpu, part_ref in ((tw.real, exact.real), (tw.imag, exact.imag)):
            ulp = np.spacing(np.abs(part_ref).astype(np.float32)).astype(np.float64)
            err = np.abs(part_gpu.astype(np.float64) - part_ref)
            assert np.all(err <= ulp + 1e-15), np.max(err - ulp)
        plan.close()


def test_large_plans_refused_where_one_signal_must_fit():
    M, s = 18, 15
    rng = rng_for(4106, 0)
    plan = native.Plan(M, homogeneous_support(M, s, rng).J.tolist())
    k = plan.k
    x = torch.zeros((2, k), dtype=torch.complex64, device="cuda")
    y = torch.zeros_like(x)

    def status(fn):
        with pytest.raises(native.HiDFTError) as ei:
            fn()
        return ei.value.status_name

    cfg = native.ExecConfig(native.PREC_FP32, native.SCHED_SHORT_LAST, 16, 0)
    assert status(lambda: plan.execute_ptr(x.data_ptr(), k, y.data_ptr(), k, 2, config=cfg)) == \
        "HIDFT_ERR_UNSUPPORTED"
    assert status(lambda: plan.execute_ptr(x.data_ptr(), k, y.data_ptr(), k, 2, plain=True)) == \
        "HIDFT_ERR_UNSUPPORTED"
    assert status(lambda: native.Group([(plan, x.data_ptr(), k, y.data_ptr(), k, 2)])) == \
        "HIDFT_ERR_UNSUPPORTED"
    assert status(lambda: plan.autotune_ptr(x.data_ptr(), k, y.data_ptr(), k, 2, reps=1)) == \
        "HIDFT_ERR_UNSUPPORTED"
    wb = plan.workspace_bytes(2)
    work = torch.empty(wb // 8 + 8, dtype=torch.complex64, device="cuda")
    # too small, missing, misaligned, overlapping
    assert status(lambda: plan.execute_ws_ptr(x.data_ptr(), k, y.data_ptr(), k, 2,
                                              work.data_ptr(), wb - 8)) == "HIDFT_ERR_INVALID_ARGUMENT"
    assert status(lambda: plan.execute_ws_ptr(x.data_ptr(), k, y.data_ptr(), k, 2, 0, wb)) == \
        "HIDFT_ERR_INVALID_ARGUMENT"
    assert status(lambda: plan.execute_ws_ptr(x.data_ptr(), k, y.data_ptr(), k, 2,
                                              work.data_ptr() + 4, wb)) == "HIDFT_ERR_INVALID_ARGUMENT"
    assert status(lambda: plan.execute_ws_ptr(x.data_ptr(), k, y.data_ptr(), k, 2,
                                              y.data_ptr(), wb)) == "HIDFT_ERR_INVALID_ARGUMENT"
    # the inverse map's workspace is checked the same way
    assert status(lambda: plan.inverse_ws_ptr(x.data_ptr(), k, y.data_ptr(), k, 2,
                                              work.data_ptr(), wb - 8)) == "HIDFT_ERR_INVALID_ARGUMENT"
    assert status(lambda: plan.inverse_ws_ptr(x.data_ptr(), k, y.data_ptr(), k, 2, 0, wb)) == \
        "HIDFT_ERR_INVALID_ARGUMENT"
    assert status(lambda: plan.inverse_ws_ptr(x.data_ptr(), k, y.data_ptr(), k, 2,
                                              work.data_ptr() + 4, wb)) == "HIDFT_ERR_INVALID_ARGUMENT"
    assert status(lambda: plan.inverse_ws_ptr(x.data_ptr(), k, y.data_ptr(), k, 2,
                                              x.data_ptr(), wb)) == "HIDFT_ERR_INVALID_ARGUMENT"
    # the single-pass sizes need no workspace
    small = native.Plan(12, homogeneous_support(12, 10, rng).J.tolist())
    assert small.workspace_bytes(1000) == 0
    small.close()
    plan.close()


@pytest.mark.parametrize("M,s", [(20, 15), (22, 17), (24, 20), (24, 21), (24, 22)])
def test_large_inverse_against_oracle(M, s):
    rng = rng_for(4107, s)
    plan = native.Plan(M, homogeneous_support(M, s, rng).J.tolist())
    k = plan.k
    J = homogeneous_support(M, s, rng_for(4107, s)).J.tolist()
    I = plan.samples().tolist()
    c = complex_normal((2, k), rng).astype(np.complex64)
    want = oracle.synthesize_samples_fft(M, J, c.astype(np.complex128), I)
    xc = torch.from_numpy(c).cuda()
    f = torch.full_like(xc, complex(np.nan, np.nan))
    plan.inverse_ptr(xc.data_ptr(), k, f.data_ptr(), k, 2)
    torch.cuda.synchronize()
    got = f.cpu().numpy().astype(np.complex128)
    err = oracle.rel_l2(got, want)
    _say(f"large inverse: M={M} s={s}, every sample against the oracle, rel-L2 {np.max(err):.3e}")
    assert np.max(err) <= TOL, err
    # the caller's workspace gives the same bits; in place too
    wb = plan.workspace_bytes(2)
    work = torch.empty(wb // 8, dtype=torch.complex64, device="cuda")
    g = torch.full_like(xc, complex(np.nan, np.nan))
    plan.inverse_ws_ptr(xc.data_ptr(), k, g.data_ptr(), k, 2, work.data_ptr(), wb)
    h = xc.clone()
    plan.inverse_ws_ptr(h.data_ptr(), k, h.data_ptr(), k, 2, work.data_ptr(), wb)
    torch.cuda.synchronize()
    assert torch.equal(g, f) and torch.equal(h, f)
    # forward after inverse: the coefficients back
    back = plan.execute(f)
    torch.cuda.synchronize()
    rt = oracle.rel_l2(back.cpu().numpy().astype(np.complex128), c.astype(np.complex128))
    assert np.max(rt) <= 2 * TOL, rt
    plan.close()
