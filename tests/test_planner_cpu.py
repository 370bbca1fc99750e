"""Host planner (C ABI, HOST_ONLY plans) against the FP64 oracle, bit-exact.

These run on the CPU: the planner is host code and HOST_ONLY plans make no HIP
call.  No compute runs on a device here.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from workloads import composite_support, elementary_support, homogeneous_support, rng_for

native = pytest.importorskip("paper_2211_15299_amd.native")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "hidft.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hidft_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = native.lib()
    names = _header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    bound = {n for n, _, _ in native.SIGNATURES}
    assert set(names) == bound, set(names) ^ bound


def _random_cases(config, n, max_M=24, max_s=12):
    for seed in range(n):
        rng = rng_for(config, seed)
        M = int(rng.integers(0, max_M + 1))
        s = int(rng.integers(0, min(M, max_s) + 1))
        yield M, homogeneous_support(M, s, rng)


def test_planner_matches_oracle_bit_exactly():
    for M, sup in _random_cases(1001, 150):
        J = sup.J.tolist()
        plan = native.Plan(M, J, host_only=True)
        r = oracle.pivots(M, J)
        assert plan.pivots() == r == list(sup.levels)
        assert plan.s == len(r) and plan.k == len(J)
        assert plan.samples().tolist() == oracle.sample_set(M, J)
        fp, num, den = plan.schedule()
        assert fp.tolist() == oracle.frequency_positions(M, J)
        tw = oracle.twiddle_exponents(M, J)
        assert num.tolist() == [m for (_, _, m, _) in tw]
        assert den.tolist() == [ru for (_, _, _, ru) in tw]
        piv, hom = native.analyze(M, J)
        assert piv == r and hom


def test_planner_bit_exact_over_ten_thousand_generator_sets():
    """10^4 seeded homogeneous supports (N <= 2^16, k <= 64): pivots, sample
    set I_r, frequency positions and twiddle exponents equal the oracle's."""
    for seed in range(10_000):
        rng = rng_for(1010, seed)
        M = int(rng.integers(0, 17))
        s = int(rng.integers(0, min(M, 6) + 1))
        sup = homogeneous_support(M, s, rng)
        J = sup.J.tolist()
        plan = native.Plan(M, J, host_only=True)
        r = oracle.pivots(M, J)
        assert plan.pivots() == r == list(sup.levels), (seed, M, J)
        assert plan.samples().tolist() == oracle.sample_set(M, J), (seed, M, J)
        fp, num, den = plan.schedule()
        assert fp.tolist() == oracle.frequency_positions(M, J), (seed, M, J)
        tw = oracle.twiddle_exponents(M, J)
        assert num.tolist() == [m for (_, _, m, _) in tw], (seed, M, J)
        assert den.tolist() == [ru for (_, _, _, ru) in tw], (seed, M, J)


def test_planner_at_large_k_and_N():
    for M, s in [(63, 10), (40, 14), (24, 16), (20, 12)]:
        sup = homogeneous_support(M, s, rng_for(1002, M))
        J = sup.J.tolist()
        plan = native.Plan(M, J, host_only=True)
        assert plan.pivots() == list(sup.levels)
        samples = plan.samples()
        assert len(set(samples.tolist())) == len(J)
        assert np.all(samples[1:] > samples[:-1])
        if s <= 12:
            assert plan.samples().tolist() == oracle.sample_set(M, J)
            fp, num, den = plan.schedule()
            assert fp.tolist() == oracle.frequency_positions(M, J)
            assert num.tolist() == [m for (_, _, m, _) in oracle.twiddle_exponents(M, J)]


def test_analyze_matches_oracle_on_arbitrary_sets():
    """Non-homogeneous and non-power-of-two sets: pivots and verdict agree."""
    for seed in range(200):
        rng = rng_for(1003, seed)
        M = int(rng.integers(1, 12))
        k = int(rng.integers(1, min(1 << M, 40) + 1))
        J = rng.choice(1 << M, size=k, replace=False).tolist()
        piv, hom = native.analyze(M, J)
        assert piv == oracle.pivots(M, J)
        assert hom == oracle.is_homogeneous(M, J)


def test_exhaustive_small_sets():
    """Every subset of Z_16: analyze agrees with the oracle's definitions."""
    import itertools
    M = 4
    for size in range(1, 17):
        for J in itertools.combinations(range(16), size):
            piv, hom = native.analyze(M, list(J))
            assert piv == oracle.pivots(M, list(J))
            assert hom == oracle.is_homogeneous(M, list(J))


def test_pivots_invariant_under_odd_dilation_and_translation():
    for seed in range(50):
        rng = rng_for(1004, seed)
        M = int(rng.integers(2, 30))
        k = int(rng.integers(2, 64))
        if k > (1 << M):
            continue
        J = np.unique(rng.integers(0, 1 << M, size=k, dtype=np.uint64))
        d = int(rng.integers(0, 1 << (M - 1))) * 2 + 1
        t = int(rng.integers(0, 1 << M))
        J2 = [((int(j) * d + t) % (1 << M)) for j in J]
        assert native.analyze(M, J.tolist())[0] == native.analyze(M, J2)[0]


hypothesis = pytest.importorskip("hypothesis")
st = hypothesis.strategies


@hypothesis.settings(max_examples=300, deadline=None, derandomize=True)
@hypothesis.given(data=st.data(), M=st.integers(1, 40))
def test_affine_invariance_property(data, M):
    """Pivots, the homogeneity verdict and the sample set are unchanged by an
    odd dilation and a translation of J, for arbitrary sets drawn by
    hypothesis: two leaves first meet at the level given by the 2-adic
    valuation of their difference (Sec. VI), which both maps preserve."""
    N = 1 << M
    J = data.draw(st.lists(st.integers(0, N - 1), min_size=1, max_size=48, unique=True))
    d = data.draw(st.integers(0, (N >> 1) - 1 if M > 1 else 0)) * 2 + 1
    t = data.draw(st.integers(0, N - 1))
    J2 = [(j * d + t) % N for j in J]
    piv, hom = native.analyze(M, J)
    piv2, hom2 = native.analyze(M, J2)
    assert piv == piv2 == oracle.pivots(M, J2)
    assert hom == hom2 == oracle.is_homogeneous(M, J)
    if hom and len(J) > 1:
        assert (native.Plan(M, J, host_only=True).samples().tolist()
                == native.Plan(M, J2, host_only=True).samples().tolist())


def test_special_families_and_composites():
    rng = rng_for(1005, 0)
    sup = elementary_support(10, 6, rng)
    plan = native.Plan(10, sup.J.tolist(), host_only=True)
    assert plan.pivots() == list(range(6))
    assert plan.samples().tolist() == [b << 4 for b in range(64)]
    comp = composite_support(24, [(0, 8, 4), (10, 10, 5), (21, 3, 2)], rng)
    plan = native.Plan(24, comp.J.tolist(), host_only=True)
    assert plan.pivots() == list(comp.levels)
    assert plan.samples().tolist() == oracle.sample_set(24, comp.J.tolist())
    # J = Z_N and k = 1
    plan = native.Plan(5, list(range(32)), host_only=True)
    assert plan.samples().tolist() == list(range(32))
    plan = native.Plan(7, [77], host_only=True)
    assert plan.k == 1 and plan.s == 0 and plan.samples().tolist() == [0]
    plan = native.Plan(0, [0], host_only=True)
    assert plan.k == 1


@pytest.mark.parametrize("M,J,status", [
    (10, [0, 512, 1, 6, 7], "HIDFT_ERR_SIZE_NOT_POW2"),          # Sec. IX example
    (4, [1, 2, 4, 8], "HIDFT_ERR_NOT_HOMOGENEOUS"),             # Sec. X, J*
    (10, [1, 2, 3, 1024], "HIDFT_ERR_INDEX_OUT_OF_RANGE"),
    (10, [5, 6, 5, 7], "HIDFT_ERR_DUPLICATE_INDEX"),
    (64, [0], "HIDFT_ERR_INVALID_ARGUMENT"),
    (2, [0, 1, 2, 3, 4], "HIDFT_ERR_INVALID_ARGUMENT"),         # k > N
    (30, np.arange(1 << 23, dtype=np.uint64), "HIDFT_ERR_UNSUPPORTED"),  # device plan above 2^22
])
def test_plan_create_rejects(M, J, status):
    with pytest.raises(native.HiDFTError) as ei:
        native.Plan(M, J, host_only=(status != "HIDFT_ERR_UNSUPPORTED"))
    assert ei.value.status_name == status
    assert native.lib().hidft_last_error()


def test_perturbed_homogeneous_sets_are_rejected():
    n_rej = 0
    for seed in range(60):
        rng = rng_for(1006, seed)
        M = int(rng.integers(5, 16))
        s = int(rng.integers(2, min(M - 2, 8) + 1))
        J = homogeneous_support(M, s, rng).J.tolist()
        free = sorted(set(range(1 << M)) - set(J)) if M <= 12 else None
        j_new = free[int(rng.integers(0, len(free)))] if free else int(rng.integers(0, 1 << M))
        if j_new in J:
            continue
        J2 = list(J)
        J2[0] = j_new
        want_hom = oracle.is_homogeneous(M, J2)
        if want_hom:
            native.Plan(M, J2, host_only=True)
        else:
            n_rej += 1
            with pytest.raises(native.HiDFTError) as ei:
                native.Plan(M, J2, host_only=True)
            assert ei.value.status_name == "HIDFT_ERR_NOT_HOMOGENEOUS"
    assert n_rej > 30


def test_null_and_bad_arguments():
    L = native.lib()
    out = ctypes.c_void_p(None)
    assert L.hidft_plan_create(4, None, 4, native.HIDFT_PLAN_HOST_ONLY, None, ctypes.byref(out)) == 1
    J = (ctypes.c_uint64 * 2)(0, 1)
    assert L.hidft_plan_create(4, J, 2, 0x80, None, ctypes.byref(out)) == 1
    assert L.hidft_plan_create(4, J, 2, native.HIDFT_PLAN_HOST_ONLY, None, None) == 1
    assert L.hidft_analyze(4, J, 0, None, None, None) == 1
    assert L.hidft_plan_destroy(None) == 0
    assert L.hidft_plan_get_pivots(None, None) == 1
    assert L.hidft_execute(None, None, 0, None, 0, 1, None) == 1
    plan = native.Plan(4, [0, 1], host_only=True)
    # execute on a HOST_ONLY plan is refused before any HIP call
    assert L.hidft_execute(plan.handle, None, 2, None, 2, 1, None) == 1
    assert "HOST_ONLY" in L.hidft_last_error().decode()
    for st in range(9):
        assert native.status_string(st) == native.STATUS_NAMES[st]
