"""GPU parity of the execution variants (hidft_execute_config) against the FP64
oracle.

Variants: the two groupings of the stages (short group first or last) in
FP32, radix-16 or radix-32 groups, and the first group (radix 16, or radix 32
for k >= 2^13) on the matrix cores with a two-term FP16 or three-term BF16
split (FP32 accumulation).  Every variant must meet the
same bar as the default path, rel-L2 <= 1e-5 per transform; the launch shape
(blocks per CU) must not change a single bit.
"""
import sys

import numpy as np
import pytest

import oracle
from tests.positions import positions_vs_oracle
from workloads import (complex_normal, homogeneous_support, log_uniform_coefficients, rng_for,
                       sample_values)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2211_15299_amd.native")

TOL = 1e-5
FP32, F16X2, BF16X3 = native.PREC_FP32, native.PREC_F16X2, native.PREC_BF16X3
DEFAULT, FIRST, LAST = native.SCHED_DEFAULT, native.SCHED_SHORT_FIRST, native.SCHED_SHORT_LAST


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


def _variants(s):
    """(precision, schedule, radix) of every variant of size 2^s."""
    out = [(FP32, FIRST, 16), (FP32, LAST, 16)]
    if s >= 4:
        out += [(F16X2, DEFAULT, 0), (BF16X3, DEFAULT, 0)]
    if s >= 13:
        out += [(FP32, FIRST, 32), (FP32, LAST, 32), (F16X2, DEFAULT, 32), (BF16X3, LAST, 32)]
    return out


def _run(plan, f, cfg, ld_in=None, ld_out=None):
    batch, k = f.shape
    ld_in = ld_in or k
    ld_out = ld_out or k
    x = torch.zeros((batch, ld_in), dtype=torch.complex64, device="cuda")
    x[:, :k] = torch.from_numpy(np.ascontiguousarray(f).astype(np.complex64))
    y = torch.full((batch, ld_out), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
    plan.execute_ptr(x.data_ptr(), ld_in, y.data_ptr(), ld_out, batch, config=cfg)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    assert np.all(np.isnan(out[:, k:])), "wrote past k in the output rows"
    return out[:, :k].astype(np.complex128)


def _check(got, want, label, tol=TOL):
    err = oracle.rel_l2(got, want)
    mabs = oracle.max_abs(got, want)
    _say(f"{label}: rel-L2 max {np.max(err):.3e} mean {np.mean(err):.3e} "
         f"max-abs {np.max(mabs):.3e}")
    assert np.all(np.isfinite(got)), label
    assert np.max(err) <= tol, label
    return err


@pytest.mark.parametrize("s", list(range(1, 15)))
def test_variants_every_size(s):
    """Every variant of every size against the oracle; ragged batches (not a
    multiple of the signals per block or of the grid), strided rows."""
    rng = rng_for(2100, s)
    M = int(rng.integers(max(s, 1), 25))
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    k = len(J)
    batch = 3 if s >= 12 else 37
    plan = native.Plan(M, J)
    I = plan.samples().tolist()
    assert I == sorted(oracle.sample_pattern_recursive(M, sup.levels))
    f = sample_values(M, k, batch, rng)
    rows = list(range(batch)) if k <= 1024 else [0, batch - 1]
    want = oracle.adjoint_coefficients(M, J, I, f[rows])
    for prec, sched, radix in _variants(s):
        _say(f"case s={s} M={M} prec={prec} sched={sched} radix={radix}")
        base = _run(plan, f, native.ExecConfig(prec, sched, radix, 0), ld_in=k + 3,
                    ld_out=k + 5)
        _check(base[rows], want, f"s={s} prec={prec} sched={sched} radix={radix}")
        for bpc in (1, 2):
            again = _run(plan, f, native.ExecConfig(prec, sched, radix, bpc))
            assert np.array_equal(again, base), f"blocks_per_cu={bpc} changed the result"
    plan.close()


def test_default_config_is_hidft_execute():
    rng = rng_for(2101, 0)
    M, s = 20, 11
    sup = homogeneous_support(M, s, rng)
    plan = native.Plan(M, sup.J.tolist())
    f = sample_values(M, plan.k, 40, rng)
    x = torch.from_numpy(f.astype(np.complex64)).cuda()
    a = plan.execute(x)
    b = plan.execute(x, config=native.ExecConfig(FP32, DEFAULT, 0, 0))
    c = plan.execute(x, config=native.ExecConfig(FP32, LAST, 0, 0))
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_config2_full_size_matrix_cores():
    """N = 2^20, k = 2^12, 4096 signals: both split precisions at full size on
    sampled transforms, and close to the FP32 path on every transform."""
    rng = rng_for(2, 0)
    M, s, batch = 20, 12, 4096
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    plan = native.Plan(M, J)
    f = sample_values(M, plan.k, batch, rng)
    rows = sorted(set([0, batch - 1] + rng.choice(batch, 10, replace=False).tolist()))
    want = oracle.adjoint_coefficients(M, J, plan.samples().tolist(), f[rows])
    ref = _run(plan, f, native.ExecConfig(FP32, DEFAULT, 0, 0))
    for prec in (F16X2, BF16X3):
        _say(f"C2 prec={prec}")
        got = _run(plan, f, native.ExecConfig(prec, DEFAULT, 0, 0))
        _check(got[rows], want, f"C2 prec={prec} sampled")
        _check(got, ref, f"C2 prec={prec} vs FP32 (all 4096)", tol=2 * TOL)


@pytest.mark.parametrize("prec,radix", [(F16X2, 16), (BF16X3, 16), (F16X2, 32), (BF16X3, 32)])
def test_config4_precision_matrix_cores(prec, radix):
    """N = 2^22, k = 2^14, 1024 signals, |c| log-uniform on [1e-3, 1e3] with
    random phase: per-instance error against the seeded coefficients, with
    the radix-16 or radix-32 first group on the matrix cores."""
    rng = rng_for(4, 0)
    M, s, batch = 22, 14, 1024
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    k = len(J)
    plan = native.Plan(M, J)
    I = plan.samples().tolist()
    n_exact = 8
    c = log_uniform_coefficients((n_exact, k), rng)
    _say(f"C4 prec={prec} radix={radix}: synthesising {n_exact} signals with the oracle")
    f_exact = oracle.synthesize_samples_fft(M, J, c, I)
    f = np.empty((batch, k), dtype=np.complex128)
    f[:n_exact] = f_exact
    scale = np.sqrt(np.mean(np.abs(f_exact) ** 2))
    f[n_exact:] = complex_normal((batch - n_exact, k), rng, scale=scale)
    got = _run(plan, f, native.ExecConfig(prec, DEFAULT, radix, 0))
    _check(got[:n_exact], c, f"C4 prec={prec} radix={radix} seeded recovery")
    ref = _run(plan, f, native.ExecConfig(FP32, DEFAULT, 0, 0))
    _check(got, ref, f"C4 prec={prec} radix={radix} vs FP32 (all 1024)", tol=2 * TOL)
    per_row = positions_vs_oracle(M, J, I, f, got, 64, rng_for(4, 2))
    _say(f"C4 prec={prec} radix={radix}: all {batch} transforms on 64 positions each "
         f"against the oracle: rel-L2 max {per_row.max():.3e}")
    assert per_row.max() <= TOL


def test_split_precision_dynamic_range():
    """The FP16 split scales each 16-value column by a power of two: rows of
    zeros, of tiny and of huge magnitude, and rows mixing 1e-20 and 1e20,
    all match the FP32 path relative to the row's norm."""
    rng = rng_for(2102, 0)
    M, s = 14, 8
    sup = homogeneous_support(M, s, rng)
    plan = native.Plan(M, sup.J.tolist())
    k = plan.k
    base = complex_normal((6, k), rng)
    f = np.zeros((8, k), dtype=np.complex128)
    f[1] = base[0] * 1e-30
    f[2] = base[1] * 1e30
    f[3] = base[2] * np.where(rng.random(k) < 0.5, 1e-20, 1e20)
    f[4] = base[3]
    f[4, ::7] = 0
    f[5] = base[4] * 10.0 ** rng.uniform(-6, 6, k)
    f[6, 17] = 3.0 - 4.0j                      # a single nonzero sample
    f[7] = base[5] * 65504.0                   # the largest FP16 magnitude
    ref = _run(plan, f, native.ExecConfig(FP32, DEFAULT, 0, 0))
    assert np.all(ref[0] == 0)
    for prec in (F16X2, BF16X3):
        got = _run(plan, f, native.ExecConfig(prec, DEFAULT, 0, 0))
        assert np.all(got[0] == 0), "zero samples must give zero coefficients"
        _check(got[1:], ref[1:], f"dynamic range prec={prec}", tol=2 * TOL)
        # the single sample: every coefficient has modulus (N/k) * 5
        assert np.allclose(np.abs(got[6]), (2.0 ** M / k) * 5.0, rtol=1e-5)


def test_split_precision_dynamic_range_radix32():
    """The radix-32 matrix-core group scales each 32-value column (two
    16-value halves in different operands) by one power of two: a column
    whose halves differ by 40 orders of magnitude, zeros and huge rows."""
    rng = rng_for(2104, 0)
    M, s = 16, 13
    sup = homogeneous_support(M, s, rng)
    plan = native.Plan(M, sup.J.tolist())
    k = plan.k
    base = complex_normal((4, k), rng)
    f = np.zeros((5, k), dtype=np.complex128)
    f[1] = base[0] * 1e30
    # group 1 works on columns a = col + c 2^{s-5}, c < 32; its halves c < 16
    # and c >= 16 are the positions a < k/2 and a >= k/2
    f[2] = base[1] * np.where(np.arange(k) < k // 2, 1e-20, 1e20)
    f[3] = base[2] * 10.0 ** rng.uniform(-6, 6, k)
    f[4] = base[3]
    ref = _run(plan, f, native.ExecConfig(FP32, DEFAULT, 0, 0))
    for prec in (F16X2, BF16X3):
        got = _run(plan, f, native.ExecConfig(prec, DEFAULT, 32, 0))
        assert np.all(got[0] == 0), "zero samples must give zero coefficients"
        _check(got[1:], ref[1:], f"dynamic range radix 32 prec={prec}", tol=2 * TOL)


def test_variant_errors():
    rng = rng_for(2103, 0)
    small = native.Plan(12, homogeneous_support(12, 3, rng).J.tolist())   # k = 8
    odd = native.Plan(16, homogeneous_support(16, 9, rng).J.tolist())     # s = 9
    x = torch.zeros((2, 512), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)

    def status(plan, cfg):
        try:
            plan.execute_ptr(x.data_ptr(), plan.k, y.data_ptr(), plan.k, 2, config=cfg)
        except native.HiDFTError as e:
            return e.status_name
        return "HIDFT_OK"

    assert status(small, native.ExecConfig(F16X2, DEFAULT, 0, 0)) == "HIDFT_ERR_UNSUPPORTED"
    assert status(small, native.ExecConfig(BF16X3, LAST, 0, 0)) == "HIDFT_ERR_UNSUPPORTED"
    assert status(small, native.ExecConfig(FP32, LAST, 0, 0)) == "HIDFT_OK"
    assert status(odd, native.ExecConfig(F16X2, FIRST, 0, 0)) == "HIDFT_ERR_UNSUPPORTED"
    assert status(odd, native.ExecConfig(F16X2, LAST, 0, 0)) == "HIDFT_OK"
    assert status(odd, native.ExecConfig(7, DEFAULT, 0, 0)) == "HIDFT_ERR_INVALID_ARGUMENT"
    assert status(odd, native.ExecConfig(FP32, 9, 0, 0)) == "HIDFT_ERR_INVALID_ARGUMENT"
    assert status(odd, native.ExecConfig(FP32, DEFAULT, 8, 0)) == "HIDFT_ERR_INVALID_ARGUMENT"
    assert status(odd, native.ExecConfig(FP32, DEFAULT, 32, 0)) == "HIDFT_ERR_UNSUPPORTED"
    assert status(odd, native.ExecConfig(FP32, DEFAULT, 16, 0)) == "HIDFT_OK"
    st = native.lib().hidft_execute_config(odd.handle, None, x.data_ptr(), 512, y.data_ptr(),
                                           512, 2, None)
    assert native.STATUS_NAMES[st] == "HIDFT_ERR_INVALID_ARGUMENT"
    torch.cuda.synchronize()
    # a 16-point plan whose s divides by 4 accepts SHORT_FIRST with the matrix cores
    p16 = native.Plan(12, homogeneous_support(12, 8, rng).J.tolist())
    assert status(p16, native.ExecConfig(BF16X3, FIRST, 0, 0)) == "HIDFT_OK"
    big = native.Plan(20, homogeneous_support(20, 13, rng).J.tolist())
    xb = torch.zeros((1, big.k), dtype=torch.complex64, device="cuda")
    yb = torch.empty_like(xb)

    def status_big(cfg):
        try:
            big.execute_ptr(xb.data_ptr(), big.k, yb.data_ptr(), big.k, 1, config=cfg)
        except native.HiDFTError as e:
            return e.status_name
        return "HIDFT_OK"

    assert status_big(native.ExecConfig(FP32, LAST, 32, 0)) == "HIDFT_OK"
    assert status_big(native.ExecConfig(F16X2, DEFAULT, 32, 0)) == "HIDFT_OK"
    assert status_big(native.ExecConfig(BF16X3, LAST, 32, 0)) == "HIDFT_OK"
    # the radix-32 matrix-core group is a full five stages: 5 divides neither 13 nor 14
    assert status_big(native.ExecConfig(F16X2, FIRST, 32, 0)) == "HIDFT_ERR_UNSUPPORTED"
    assert status(odd, native.ExecConfig(BF16X3, DEFAULT, 32, 0)) == "HIDFT_ERR_UNSUPPORTED"
    torch.cuda.synchronize()
