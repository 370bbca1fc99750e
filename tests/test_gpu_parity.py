"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar: relative L2 error <= 1e-5 per transform (FP32 arithmetic), reported with
the max-abs error.  Inputs come from the seeded generators; expected values
come only from the oracle.  Large configurations are checked in full on
sampled transforms, and every transform on 64 seeded positions of its own
(tests/positions.py) and on the energy identity ||c||^2 = (N^2/k) ||f_I||^2,
which holds for any samples because F(J, I_r) is k times a unitary matrix
(Lemma 1).
"""
import sys

import numpy as np
import pytest

import oracle
from tests.positions import positions_vs_oracle
from workloads import (complex_normal, elementary_support, homogeneous_support,
                       log_uniform_coefficients, rng_for, sample_values)

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


def _run(plan, f64, plain=False, ld_in=None, ld_out=None):
    """Upload complex64 samples (batch, k), execute, return complex128 results."""
    batch, k = f64.shape
    ld_in = ld_in or k
    ld_out = ld_out or k
    x = torch.zeros((batch, ld_in), dtype=torch.complex64, device="cuda")
    x[:, :k] = torch.from_numpy(f64.astype(np.complex64))
    y = torch.full((batch, ld_out), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
    plan.execute_ptr(x.data_ptr(), ld_in, y.data_ptr(), ld_out, batch, plain=plain)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    assert np.all(np.isnan(out[:, k:])), "wrote past k in the output rows"
    return out[:, :k].astype(np.complex128)


def _check(got, want, label, tol=TOL):
    err = oracle.rel_l2(got, want)
    mabs = oracle.max_abs(got, want)
    _say(f"{label}: rel-L2 max {np.max(err):.3e} mean {np.mean(err):.3e} max-abs {np.max(mabs):.3e}")
    assert np.all(np.isfinite(got))
    assert np.max(err) <= tol, label
    return err


def _energy_ok(c, f, M, k, tol=TOL):
    N = float(1 << M)
    lhs = np.sum(np.abs(c) ** 2, axis=-1)
    rhs = (N * N / k) * np.sum(np.abs(f.astype(np.complex128)) ** 2, axis=-1)
    rel = np.abs(lhs - rhs) / rhs
    assert np.max(rel) <= 2 * tol, np.max(rel)
    return rel


# ----------------------------------------------------------------- every size

@pytest.mark.parametrize("s", list(range(0, 15)))
def test_every_size_against_oracle(s):
    """Each k = 2^s the executor supports, a ragged batch, random homogeneous J."""
    rng = rng_for(2000, s)
    M = int(rng.integers(max(s, 1), 25))
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    k = len(J)
    batch = {0: 301, 1: 257, 2: 300, 3: 513}.get(s, 3 if s >= 12 else 37)
    _say(f"case s={s} M={M} batch={batch}")
    plan = native.Plan(M, J)
    f = sample_values(M, k, batch, rng)
    got = _run(plan, f)
    I = oracle.sample_set(M, J) if s <= 12 else plan.samples().tolist()
    if s > 12:
        assert I == sorted(oracle.sample_pattern_recursive(M, sup.levels))
    rows = range(batch) if k <= 1024 else [0, batch - 1]
    want = oracle.adjoint_coefficients(M, J, I, f[list(rows)])
    _check(got[list(rows)], want, f"s={s}")
    _energy_ok(got, f, M, k)
    plan.close()


def test_lu_route_on_midsize():
    """The dense LU solve of the paper's submatrix system, directly."""
    rng = rng_for(2001, 0)
    M, s = 18, 9
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    plan = native.Plan(M, J)
    f = sample_values(M, len(J), 5, rng)
    got = _run(plan, f)
    want = oracle.coefficients(M, J, f.astype(np.complex128), method="lu")
    _check(got, want, "lu k=512")


# ---------------------------------------------------- configuration 1 (plain)

@pytest.mark.parametrize("kind", ["elementary", "random_pivots"])
def test_config1_single_signal_recovery(kind):
    """N = 2^10, k = 64: seeded c ~ CN(0,1), signal synthesised by the oracle,
    sampled on I_r, rounded to complex64; both GPU paths recover c."""
    rng = rng_for(1, 0 if kind == "elementary" else 1)
    M, s = 10, 6
    sup = elementary_support(M, s, rng) if kind == "elementary" else homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    assert oracle.is_homogeneous(M, J)
    c = complex_normal(len(J), rng)
    I = oracle.sample_set(M, J)
    f = oracle.synthesize_samples(M, J, c, I)[None, :]
    plan = native.Plan(M, J)
    assert plan.samples().tolist() == I
    got = _run(plan, f)
    _check(got, c[None, :], f"C1 {kind} fused vs seeded c")
    got_plain = _run(plan, f, plain=True)
    _check(got_plain, c[None, :], f"C1 {kind} plain vs seeded c")
    want = oracle.solve_coefficients(M, J, I, f.astype(np.complex64).astype(np.complex128))
    _check(got, want, f"C1 {kind} fused vs LU on the complex64 samples")


# ------------------------------------------ configuration 2 (batched, full size)

def test_config2_full_size():
    """N = 2^20, k = 2^12, one J, 4096 signals in one launch (as timed)."""
    rng = rng_for(2, 0)
    M, s, batch = 20, 12, 4096
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    k = len(J)
    plan = native.Plan(M, J)
    f = sample_values(M, k, batch, rng)
    _say("C2: executing 4096 x 4096")
    got = _run(plan, f)
    I = plan.samples().tolist()
    assert I == sorted(oracle.sample_pattern_recursive(M, sup.levels))
    rows = sorted(set([0, 1, batch // 2, batch - 1] + rng.choice(batch, 12, replace=False).tolist()))
    want = oracle.adjoint_coefficients(M, J, I, f[rows])
    err = _check(got[rows], want, "C2 sampled transforms")
    _energy_ok(got, f, M, k)
    # every transform on 64 positions of its own
    per_row = positions_vs_oracle(M, J, I, f, got, 64, rng_for(2, 1))
    _say(f"C2: all {batch} transforms on 64 positions each: rel-L2 max {per_row.max():.3e}")
    assert per_row.shape == (batch,) and per_row.max() <= TOL
    # seeded-coefficient recovery for a few signals
    c = complex_normal((3, k), rng)
    fs = oracle.synthesize_samples(M, J, c, I)
    _check(_run(plan, fs), c, "C2 recovery of seeded c")
    # the plain per-signal method agrees on a slice
    got_plain = _run(plan, f[:32], plain=True)
    _check(got_plain, got[:32], "C2 plain vs fused", tol=1e-6)
    assert err.shape[0] == len(rows)


# ---------------------------------------------- configuration 4 (precision)

def test_config4_precision_fp32():
    """N = 2^22, k = 2^14, 1024 signals, |c| log-uniform on [1e-3, 1e3], FP32
    butterflies: per-instance error against the seeded coefficients."""
    rng = rng_for(4, 0)
    M, s, batch = 22, 14, 1024
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    k = len(J)
    plan = native.Plan(M, J)
    I = plan.samples().tolist()
    n_exact = 8
    c = log_uniform_coefficients((n_exact, k), rng)
    _say("C4: synthesising 3 signals with the oracle")
    f_exact = oracle.synthesize_samples_fft(M, J, c, I)
    f = np.empty((batch, k), dtype=np.complex128)
    f[:n_exact] = f_exact
    scale = np.sqrt(np.mean(np.abs(f_exact) ** 2))
    f[n_exact:] = complex_normal((batch - n_exact, k), rng, scale=scale)
    got = _run(plan, f)
    _check(got[:n_exact], c, "C4 seeded recovery (FP32)")
    _energy_ok(got, f.astype(np.complex64), M, k)
    per_row = positions_vs_oracle(M, J, I, f, got, 64, rng_for(4, 1))
    _say(f"C4: all {batch} transforms on 64 positions each: rel-L2 max {per_row.max():.3e}")
    assert per_row.max() <= TOL


# --------------------------------------------------------------- properties

def test_twiddles_are_fp64_rounded_once():
    rng = rng_for(2002, 0)
    for M, s in [(20, 12), (63, 10), (12, 12), (40, 14)]:
        sup = homogeneous_support(M, s, rng)
        plan = native.Plan(M, sup.J.tolist())
        fp, num, den = plan.schedule()
        tw = plan.twiddles()
        exact = np.exp(-1j * np.pi * (num.astype(np.float64) / np.exp2(den.astype(np.float64))))
        # correctly rounded to FP32 within one unit in the last place of the
        # exact value; 1e-15 absorbs the error of numpy's own FP64 evaluation
        for part_gpu, part_ref in ((tw.real, exact.real), (tw.imag, exact.imag)):
            ulp = np.spacing(np.abs(part_ref).astype(np.float32)).astype(np.float64)
            err = np.abs(part_gpu.astype(np.float64) - part_ref)
            assert np.all(err <= ulp + 1e-15), np.max(err - ulp)
        assert np.max(np.abs(tw - exact)) < 1e-7


def test_strides_in_place_and_determinism():
    rng = rng_for(2003, 0)
    M, s = 16, 10
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    k = len(J)
    plan = native.Plan(M, J)
    f = sample_values(M, k, 9, rng)
    want = oracle.adjoint_coefficients(M, J, plan.samples().tolist(), f)
    a = _run(plan, f, ld_in=k + 3, ld_out=k + 5)
    _check(a, want, "strided")
    b = _run(plan, f)
    assert np.array_equal(a, b), "results depend on the strides"
    x = torch.from_numpy(f.astype(np.complex64)).cuda()
    plan.execute_ptr(x.data_ptr(), k, x.data_ptr(), k, f.shape[0])
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy().astype(np.complex128), b), "in place differs"
    c = _run(plan, f)
    assert np.array_equal(b, c), "not deterministic"


def test_linearity_and_shift_law():
    """GPU(alpha f + beta g) = alpha GPU(f) + beta GPU(g); samples of f(. - a)
    give c_j exp(-2 pi i a j / N) (Lemma 2)."""
    rng = rng_for(2004, 0)
    M, s = 14, 8
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    N, k = 1 << M, len(J)
    plan = native.Plan(M, J)
    I = plan.samples().tolist()
    c = complex_normal(k, rng)
    a = int(rng.integers(0, N))
    f = oracle.synthesize_samples(M, J, c, I)
    fa = oracle.synthesize_samples(M, J, c, [(i - a) % N for i in I])
    got = _run(plan, np.stack([f, fa]))
    phase = np.exp(-2j * np.pi * ((a * np.array(J, dtype=object)) % N).astype(np.float64) / N)
    _check(got[1:2], (got[0] * phase)[None, :], "shift law", tol=3e-6)
    g = sample_values(M, k, 1, rng)[0]
    lin = _run(plan, np.stack([2.0 * f - 0.5j * g, f, g]))
    _check(lin[0:1], (2.0 * lin[1] - 0.5j * lin[2])[None, :], "linearity", tol=3e-6)


def test_execute_argument_errors():
    rng = rng_for(2005, 0)
    M, s = 12, 6
    sup = homogeneous_support(M, s, rng)
    plan = native.Plan(M, sup.J.tolist())
    k = plan.k
    x = torch.zeros((4, k), dtype=torch.complex64, device="cuda")
    y = torch.zeros((4, k), dtype=torch.complex64, device="cuda")

    def status(d_in, ld_in, d_out, ld_out, batch):
        return native.lib().hidft_execute(plan.handle, d_in, ld_in, d_out, ld_out, batch, None)

    assert status(x.data_ptr(), k, y.data_ptr(), k, 0) == 0          # empty batch
    assert status(x.data_ptr(), k - 1, y.data_ptr(), k, 4) == 1      # ld < k
    assert status(x.data_ptr() + 4, k, y.data_ptr(), k, 3) == 1      # misaligned
    assert status(x.data_ptr(), k, x.data_ptr() + 8, k, 3) == 1      # partial overlap
    assert status(x.data_ptr(), k, x.data_ptr(), k + 1, 3) == 1      # in place, other ld
    assert status(0, k, y.data_ptr(), k, 1) == 1                     # null
    assert status(x.data_ptr(), k, y.data_ptr(), k, 4) == 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("M,s", [(40, 10), (62, 10), (63, 12)])
def test_largest_N_recovery(M, s):
    """N up to 2^63 (the ABI's limit): seeded coefficients recovered from
    samples the oracle synthesised with exact modular phases; the twiddle
    arguments m / 2^d then carry more than 53 bits, which FP64 rounds far
    below FP32 resolution."""
    rng = rng_for(1, 1000 + M)
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    plan = native.Plan(M, J)
    c = complex_normal((3, len(J)), rng)
    f = oracle.synthesize_samples(M, J, c, plan.samples().tolist())
    got = _run(plan, f)
    _check(got, c, f"N=2^{M}, k=2^{s}")
    plan.close()


@pytest.mark.parametrize("M", [1, 4, 9, 12, 14])
def test_full_support_is_the_fft(M):
    """J = Z_N in a shuffled caller order (k = N, the degenerate case where
    the sample set is the whole signal): the coefficients are numpy's FFT
    of the signal, read in the caller's order."""
    rng = rng_for(2001, M)
    N = 1 << M
    J = rng.permutation(N).tolist()
    plan = native.Plan(M, J)
    assert plan.samples().tolist() == list(range(N))
    f = complex_normal((3, N), rng)
    got = _run(plan, f)
    want = np.fft.fft(f, axis=1)[:, J]
    _check(got, want, f"J = Z_N, N=2^{M}")
    plan.close()


def test_single_coefficient_at_the_largest_N():
    """k = 1 (Algorithm 1's base case): the coefficient is N f(0), here with
    N = 2^63 and the one sample at 0."""
    rng = rng_for(2002, 0)
    plan = native.Plan(63, [int(rng.integers(0, 1 << 62)) * 2 + 1])
    assert plan.samples().tolist() == [0]
    f = complex_normal((5, 1), rng) * 2.0 ** -63
    got = _run(plan, f)
    _check(got, f * 2.0 ** 63, "k = 1, N = 2^63")
    plan.close()
