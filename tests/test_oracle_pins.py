"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check uses a value the
paper prints (fixtures in tests/golden, each with its citation), a closed form,
an invariant, a textbook routine (numpy's FFT, a brute-force DFT written with
Python's cmath), or exhaustive search on tiny inputs.
"""
import cmath
import itertools
import math

import numpy as np
import pytest

import oracle
from tests.golden import fixtures
from workloads import (complex_normal, composite_support, elementary_support,
                       homogeneous_support, rng_for)


# ---------------------------------------------------------------- paper values

@pytest.mark.parametrize("ex", fixtures.paper_examples(), ids=lambda e: f"{e['kind']}-{e['J']}")
def test_paper_examples(ex):
    M, J, exp = ex["M"], ex["J"], ex["expected"]
    if ex["kind"] == "pivots":
        assert oracle.pivots(M, J) == exp, ex["cite"]
        assert oracle.pivots_by_tree(M, J) == exp, ex["cite"]
    elif ex["kind"] == "homogeneous":
        assert oracle.is_homogeneous(M, J) == bool(exp[0]), ex["cite"]
        if len(J) & (len(J) - 1) == 0:
            assert oracle.homogeneous_by_tree(M, J) == bool(exp[0]), ex["cite"]
    elif ex["kind"] == "pattern":
        assert sorted(oracle.sample_pattern_recursive(M, J)) == exp, ex["cite"]
        assert oracle.sample_pattern_closed_form(M, J) == set(exp), ex["cite"]
    elif ex["kind"] == "spectral":
        F = oracle.dft_submatrix(M, exp, J)
        G = F.conj().T @ F
        assert np.allclose(G, len(J) * np.eye(len(J)), atol=1e-12), ex["cite"]
    else:
        raise AssertionError(ex["kind"])


def test_printed_hidft_matrix_reproduces_in_plan_order():
    """Sec. VII-A item 4: the printed 2^-8-scaled F^{-1}(I, J) reproduces entry
    for entry with rows in the recursion order of I_r and columns in q order."""
    M, J = 10, [84, 305, 725, 992]
    r = oracle.pivots(M, J)
    assert r == [0, 2]
    rows = oracle.sample_pattern_recursive(M, r)
    assert rows == [0, 512, 128, 640]
    cols = sorted(J, key=lambda j: oracle.frequency_position(j, r))
    assert cols == [992, 305, 84, 725]
    A = oracle.idft_submatrix(M, rows, cols) * 2 ** 8
    printed = fixtures.printed_matrix()
    assert len(printed) == 16
    for idx, (i, j, val) in enumerate(printed):
        a, b = divmod(idx, 4)
        assert (rows[a], cols[b]) == (i, j)
        assert abs(A[a, b] - val) < 1e-4, (i, j, A[a, b], val)


# ------------------------------------------------------- exhaustive tiny cases

def _all_subsets(N, max_size):
    for size in range(1, max_size + 1):
        for J in itertools.combinations(range(N), size):
            yield list(J)


def _spectral_brute_force(M, J, patterns):
    """Is there an I, |I| = |J|, with F(I, J) scaled unitary?  (Def. spectral)

    Columns of F(I, J) are orthogonal iff sum_{i in I} omega^{i (j_a - j_b)}
    vanishes for every a != b; ``patterns[size]`` holds that sum for every I of
    the size and every difference d in Z_N.
    """
    N = 1 << M
    k = len(J)
    if k == 1:
        return True
    diffs = sorted({(a - b) % N for a in J for b in J if a != b})
    H = patterns[k][:, diffs]
    return bool(np.any(np.all(np.abs(H) < 1e-9, axis=1)))


def _patterns(M, max_size):
    N = 1 << M
    out = {}
    for size in range(2, max_size + 1):
        Is = np.array(list(itertools.combinations(range(N), size)))
        d = np.arange(N)
        out[size] = np.exp(-2j * np.pi * (Is[:, :, None] * d[None, None, :] % N) / N).sum(axis=1)
    return out


@pytest.mark.parametrize("M,max_size", [(3, 8), (4, 4)])
def test_propositions_1_2_3_exhaustive(M, max_size):
    """Prop. 1 (at least log2|J| pivots), Prop. 2 (tree form == pivot count ==
    pairwise-valuation form) and Prop. 3 (homogeneous iff spectral) over every
    J in Z_8 and every J in Z_16 with |J| <= 4."""
    patterns = _patterns(M, max_size)
    n_hom = 0
    for J in _all_subsets(1 << M, max_size):
        P = oracle.pivots(M, J)
        assert len(P) >= math.log2(len(J)) - 1e-12                      # Prop. 1
        assert P == oracle.pivots_by_tree(M, J)
        e_ab = {oracle.nu2(a - b) for a in J for b in J if a != b}       # Prop. 2(4)
        assert set(P) == e_ab
        hom = oracle.is_homogeneous(M, J)
        if oracle.is_power_of_two(len(J)):
            assert hom == oracle.homogeneous_by_tree(M, J)                # Prop. 2(2)
        assert hom == _spectral_brute_force(M, J, patterns)               # Prop. 3
        n_hom += hom
    assert n_hom > 0


def test_lemma1_aliasing_pattern_zeros():
    """Lemma 1: the aliasing pattern of I_r vanishes on every difference of two
    distinct elements of an r-homogeneous J (so F(J, I_r) is scaled unitary)."""
    for seed in range(30):
        rng = rng_for(900, seed)
        M = int(rng.integers(4, 12))
        s = int(rng.integers(1, min(M, 6) + 1))
        sup = homogeneous_support(M, s, rng)
        J = sup.J.tolist()
        I = oracle.sample_set(M, J)
        N = 1 << M
        for a in J[:8]:
            for b in J[:8]:
                if a != b:
                    h = sum(cmath.exp(-2j * math.pi * (i * ((a - b) % N) % N) / N) for i in I)
                    assert abs(h) < 1e-9
        F = oracle.dft_submatrix(M, J, I)
        assert np.allclose(F @ F.conj().T, len(J) * np.eye(len(J)), atol=1e-9)


# ------------------------------------------- generator pivots and the predicate

def test_generator_levels_are_the_pivots():
    """The split levels a set was constructed with are its pivot set."""
    for seed in range(60):
        rng = rng_for(901, seed)
        M = int(rng.integers(1, 20))
        s = int(rng.integers(0, min(M, 8) + 1))
        sup = homogeneous_support(M, s, rng)
        J = sup.J.tolist()
        assert oracle.pivots(M, J) == list(sup.levels)
        assert oracle.is_homogeneous(M, J)
        if M <= 12:
            assert oracle.homogeneous_by_tree(M, J)


def test_predicate_rejects_perturbed_sets():
    """Moving one element of a homogeneous set to an unused index breaks homogeneity
    (the size stays a power of two) unless the result is again homogeneous by
    the tree criterion: both predicates must agree either way."""
    for seed in range(40):
        rng = rng_for(902, seed)
        M = int(rng.integers(4, 10))
        s = int(rng.integers(1, min(M - 1, 5) + 1))
        J = homogeneous_support(M, s, rng).J.tolist()
        free = sorted(set(range(1 << M)) - set(J))
        J2 = list(J)
        J2[int(rng.integers(0, len(J)))] = free[int(rng.integers(0, len(free)))]
        assert oracle.is_homogeneous(M, J2) == oracle.homogeneous_by_tree(M, J2)


def test_special_families():
    """Sec. VI/VII-A: {0..2^s-1} has pivots 0..s-1 (elementary, uniform I);
    the periodic set has pivots M-s..M-1 and I = {0..2^s-1}; Z_N gives I = Z_N."""
    for M, s in [(6, 3), (10, 6), (12, 4)]:
        N = 1 << M
        J = list(range(1 << s))
        assert oracle.pivots(M, J) == list(range(s))
        assert oracle.sample_set(M, J) == [b << (M - s) for b in range(1 << s)]
        Jp = [b * (N >> s) for b in range(1 << s)]
        assert oracle.pivots(M, Jp) == list(range(M - s, M))
        assert oracle.sample_set(M, Jp) == list(range(1 << s))
    assert oracle.sample_set(5, list(range(32))) == list(range(32))


def test_sample_pattern_is_homogeneous_with_mirrored_pivots():
    """Sec. VII: |I_r| = 2^s, elements distinct, and I_r is (M-1-r)-homogeneous."""
    for seed in range(30):
        rng = rng_for(903, seed)
        M = int(rng.integers(2, 16))
        s = int(rng.integers(1, min(M, 7) + 1))
        r = sorted(rng.choice(M, size=s, replace=False).tolist())
        I = oracle.sample_pattern_recursive(M, r)
        assert len(set(I)) == 1 << s
        assert oracle.pivots(M, I) == sorted(M - 1 - x for x in r)


# --------------------------------------------------------- coefficient pins

def _brute_dft_on(M, f_full, J):
    """(Ff)(j) = sum_n f(n) exp(-2 pi i j n / N), written out with cmath."""
    N = 1 << M
    return [sum(f_full[n] * cmath.exp(-2j * math.pi * ((j * n) % N) / N) for n in range(N)) for j in J]


@pytest.mark.parametrize("seed", range(6))
def test_recovery_against_full_fft_and_brute_force(seed):
    """Seeded c on J -> full signal by numpy's inverse FFT -> samples on I_r ->
    oracle solve returns c; numpy's forward FFT and a brute-force DFT agree."""
    rng = rng_for(904, seed)
    M = int(rng.integers(4, 11))
    s = int(rng.integers(1, min(M, 6) + 1))
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    N = 1 << M
    c = complex_normal(len(J), rng)
    C = np.zeros(N, dtype=np.complex128)
    C[J] = c
    f_full = np.fft.ifft(C)                      # (1/N) sum c_j e^{+2 pi i jn/N}
    I = oracle.sample_set(M, J)
    f_I = f_full[I]
    assert np.allclose(oracle.synthesize_samples(M, J, c, I), f_I, atol=1e-14)
    for method in ("lu", "adjoint"):
        got = oracle.coefficients(M, J, f_I, method=method)
        assert oracle.rel_l2(got, c) < 1e-12, method
    assert np.allclose(np.fft.fft(f_full)[J], c, atol=1e-12)
    if N <= 256:
        bf = np.array(_brute_dft_on(M, f_full, J))
        assert oracle.rel_l2(bf, c) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_fft_synthesis_equals_the_direct_sum(seed):
    """synthesize_samples_fft (one inverse FFT per signal) against the direct
    O(k |I|) sum and, on tiny N, a brute-force inverse DFT written out."""
    rng = rng_for(905, seed)
    M = int(rng.integers(3, 13))
    s = int(rng.integers(1, min(M, 8) + 1))
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    N = 1 << M
    c = complex_normal((3, len(J)), rng)
    I = oracle.sample_set(M, J)
    fast = oracle.synthesize_samples_fft(M, J, c, I)
    assert fast.shape == (3, len(I))
    assert np.max(np.abs(fast - oracle.synthesize_samples(M, J, c, I))) < 1e-13
    assert np.allclose(oracle.synthesize_samples_fft(M, J, c[0], I), fast[0], atol=0)
    if N <= 64:
        brute = [[sum(c[b, t] * cmath.exp(2j * math.pi * ((J[t] * i) % N) / N)
                      for t in range(len(J))) / N for i in I] for b in range(3)]
        assert np.max(np.abs(fast - np.array(brute))) < 1e-13
    with pytest.raises(ValueError):
        oracle.synthesize_samples_fft(M, [0, 0], c[0, :2], I)


def test_full_support_is_the_fft():
    """Sec. VIII: J = Z_N reduces the Hi-DFT to the DFT (I_r = Z_N)."""
    rng = rng_for(905, 0)
    for M in (3, 5, 7):
        N = 1 << M
        f = complex_normal(N, rng)
        J = list(range(N))
        got = oracle.coefficients(M, J, f, method="lu")
        assert oracle.rel_l2(got, np.fft.fft(f)) < 1e-12


def test_energy_shift_and_linearity():
    """||c||^2 = (N^2/k) ||f_I||^2;  Lemma 2: samples of f(. - a) give
    c_j omega^{a j};  the map samples -> coefficients is linear."""
    for seed in range(10):
        rng = rng_for(906, seed)
        M = int(rng.integers(5, 16))
        s = int(rng.integers(1, min(M, 7) + 1))
        sup = homogeneous_support(M, s, rng)
        J = sup.J.tolist()
        N, k = 1 << M, len(J)
        I = oracle.sample_set(M, J)
        c = complex_normal(k, rng)
        f_I = oracle.synthesize_samples(M, J, c, I)
        assert abs(np.vdot(c, c).real - (N * N / k) * np.vdot(f_I, f_I).real) < 1e-9 * np.vdot(c, c).real
        a = int(rng.integers(0, N))
        shifted = oracle.synthesize_samples(M, J, c, [(i - a) % N for i in I])
        got = oracle.coefficients(M, J, shifted)
        want = c * np.exp(-2j * np.pi * ((a * np.array(J, dtype=object)) % N).astype(np.float64) / N)
        assert oracle.rel_l2(got, want) < 1e-11
        g_I = complex_normal(k, rng) * np.sqrt(k) / N
        lhs = oracle.coefficients(M, J, 2.5 * f_I - 1j * g_I)
        rhs = 2.5 * oracle.coefficients(M, J, f_I) - 1j * oracle.coefficients(M, J, g_I)
        assert oracle.rel_l2(lhs, rhs) < 1e-11


def test_lu_and_adjoint_agree_at_larger_k():
    rng = rng_for(907, 0)
    sup = homogeneous_support(20, 9, rng)
    J = sup.J.tolist()
    f = complex_normal((3, len(J)), rng) * np.sqrt(len(J)) / (1 << 20)
    a = oracle.coefficients(20, J, f, method="lu")
    b = oracle.coefficients(20, J, f, method="adjoint")
    assert np.max(oracle.rel_l2(a, b)) < 1e-11
    I = oracle.sample_set(20, J)
    for t in (0, 7, len(J) - 1):
        assert abs(oracle.coefficient_at(20, J[t], I, f[1], len(J)) - b[1, t]) < 1e-9 * np.abs(b[1]).max()


def test_ill_conditioned_consecutive_samples_are_avoided():
    """Sec. V-A picks I = {0..k-1}; for clustered J that system is numerically
    singular, while the system on I_r is perfectly conditioned."""
    M, J = 10, list(range(64))
    A_bad = oracle.idft_submatrix(M, list(range(64)), J)
    A_good = oracle.idft_submatrix(M, oracle.sample_set(M, J), J)
    assert np.linalg.cond(A_bad) > 1e12
    assert abs(np.linalg.cond(A_good) - 1.0) < 1e-9


# ------------------------------------------ plan orders and twiddle exponents

def _hidft_recursive(M, f_p, r, cols):
    """Algorithm 1, recursive, with the sign of Lemma 3 and f2 = second half.

    f_p: samples in recursion order of I_r; r: pivots; cols: J in q order.
    Returns F(J, I_r) f_I in q order (no normalisation).
    """
    n = len(f_p)
    if n == 1:
        return [f_p[0]] * len(cols) if len(cols) == 1 else [f_p[0]]
    half = n // 2
    left = cols[:half]
    a = f_p[:half]
    b = f_p[half:]
    X1 = _hidft_recursive(M, a, r[:-1], left)
    X2 = _hidft_recursive(M, b, r[:-1], left)
    rmax = r[-1]
    out_lo, out_hi = [], []
    for t, j in enumerate(left):
        w = cmath.exp(-2j * math.pi * (j % (1 << (rmax + 1))) / (1 << (rmax + 1)))
        out_lo.append(X1[t] + w * X2[t])
        out_hi.append(X1[t] - w * X2[t])
    return out_lo + out_hi


def _stages_from_exponents(M, k, tw, x):
    """Iterative DIT stages driven by the oracle's (u, q_lo, m, r_u) list."""
    X = np.array(x, dtype=np.complex128)
    table = {}
    for u, q_lo, m, ru in tw:
        table[(u, q_lo)] = np.exp(-1j * np.pi * m / (1 << ru))
    s = k.bit_length() - 1
    for u in range(1, s + 1):
        h = 1 << (u - 1)
        for blk in range(0, k, 2 * h):
            for q in range(h):
                w = table[(u, q)]
                P, Q = X[blk + q], X[blk + q + h]
                X[blk + q], X[blk + q + h] = P + w * Q, P - w * Q
    return X


@pytest.mark.parametrize("seed", range(8))
def test_corollary2_factorisation_pins_orders_and_twiddles(seed):
    """Corollary 2 / Lemma 3: stages built from the oracle's twiddle exponents,
    fed samples in the recursion order of I_r, yield F(J, I_r) f_I in q order;
    the recursive form of Algorithm 1 agrees; the dense product decides."""
    rng = rng_for(908, seed)
    M = int(rng.integers(3, 14))
    s = int(rng.integers(1, min(M, 7) + 1))
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    k = len(J)
    r = oracle.pivots(M, J)
    rows = oracle.sample_pattern_recursive(M, r)
    q = oracle.frequency_positions(M, J)
    assert sorted(q) == list(range(k))
    cols = [None] * k
    for t, qq in enumerate(q):
        cols[qq] = J[t]
    f = complex_normal(k, rng)
    dense = oracle.dft_submatrix(M, cols, rows) @ f
    tw = oracle.twiddle_exponents(M, J)
    assert len(tw) == k - 1
    staged = _stages_from_exponents(M, k, tw, f)
    assert np.max(np.abs(staged - dense)) < 1e-10 * np.max(np.abs(dense))
    rec = np.array(_hidft_recursive(M, list(f), r, cols))
    assert np.max(np.abs(rec - dense)) < 1e-10 * np.max(np.abs(dense))


def test_twiddle_exponent_is_well_defined():
    """All j sharing their first u-1 pivot bits agree modulo 2^{r_u}
    (homogeneity), so the twiddle does not depend on which j is used."""
    for seed in range(20):
        rng = rng_for(909, seed)
        M = int(rng.integers(3, 20))
        s = int(rng.integers(1, min(M, 7) + 1))
        J = homogeneous_support(M, s, rng).J.tolist()
        r = oracle.pivots(M, J)
        for u in range(1, s + 1):
            seen = {}
            for j in J:
                key = oracle.frequency_position(j, r) % (1 << (u - 1))
                seen.setdefault(key, set()).add(j % (1 << r[u - 1]))
            assert all(len(v) == 1 for v in seen.values())


def test_elementary_and_composite_generators_are_homogeneous():
    rng = rng_for(910, 0)
    sup = elementary_support(10, 6, rng)
    assert oracle.pivots(10, sup.J.tolist()) == list(range(6))
    comp = composite_support(16, [(0, 6, 3), (8, 8, 4)], rng)
    assert oracle.is_homogeneous(16, comp.J.tolist())
    assert oracle.pivots(16, comp.J.tolist()) == list(comp.levels)


def test_theorem1_operation_count():
    """Theorem 1: T(n) = 2 T(n+1) + 3 * 2^{s-n-1}, T(s) = 1  ->  1.5 A log A + A."""
    for s in range(0, 15):
        T = 1
        for n in range(s - 1, -1, -1):
            T = 2 * T + 3 * (1 << (s - n - 1))
        assert T == oracle.op_count(1 << s)
