"""Shift-and-Sample planner (HOST_ONLY) against the oracle's definitions."""
import numpy as np
import pytest

import oracle
from tests.golden import fixtures
from workloads import homogeneous_support, rng_for

native = pytest.importorskip("paper_2211_15299_amd.native")


def _subset(rng, M, s, frac):
    K = homogeneous_support(M, s, rng)
    keep = rng.random(len(K.J)) < frac
    J = [int(j) for j, kp in zip(K.J, keep) if kp] or [int(K.J[0])]
    return K, J


@pytest.mark.parametrize("ex", fixtures.part_homogeneous_examples(),
                         ids=lambda e: f"{e['J']}-{e['r']}")
def test_printed_examples_nodes(ex):
    M, J, r = ex["M"], ex["J"], ex["r"]
    plan = native.SASPlan(M, J, pivots=r, host_only=True)
    node_of_t, slots = plan.nodes()
    groups = {}
    for t, v in enumerate(node_of_t):
        groups.setdefault(int(v), []).append(J[t])
    assert sorted(sorted(g) for g in groups.values()) == ex["nodes"], ex["cite"]
    assert plan.mu_max == max(len(g) for g in ex["nodes"])
    rows = oracle.sas_sample_set(M, r, plan.mu_max)
    assert plan.samples().tolist() == [x for row in rows for x in row]


def test_sas_example_of_section_ix():
    """J = {0,512,1,6,7}, N = 1024 at r = (0,1): mu* = 2, 8 samples."""
    plan = native.SASPlan(10, [0, 512, 1, 6, 7], pivots=[0, 1], host_only=True)
    assert plan.mu_max == 2 and plan.samples_per_signal == 8 and plan.n_nodes == 4


def test_nodes_slots_and_samples_match_oracle():
    for seed in range(60):
        rng = rng_for(1100, seed)
        M = int(rng.integers(6, 22))
        K, J = _subset(rng, M, int(rng.integers(2, min(M, 10) + 1)), rng.uniform(0.2, 0.9))
        t = int(rng.integers(0, len(K.levels) + 1))
        r = list(K.levels[:t])
        level = (max(r) + 1) if r else 0
        mu = max(len(v) for v in oracle.level_nodes(M, J, level).values())
        # the index work of any r (weights-only plans skip the leaf-solve limits)
        plan = native.SASPlan(M, J, pivots=r, host_only=True, weights_only=True)
        assert plan.pivots() == r
        node_of_t, slots = plan.nodes()
        want = oracle.level_nodes(M, J, level)
        got = {}
        for ti, v in enumerate(node_of_t):
            got.setdefault(int(v), []).append(ti)
        assert sorted(got.values()) == sorted(want.values())
        # the slot of a node is its pivot-bit pattern
        for v, ts in got.items():
            j = J[ts[0]]
            assert slots[v] == oracle.frequency_position(j, r)
        assert plan.mu_max == mu
        rows = oracle.sas_sample_set(M, r, mu)
        assert plan.samples().tolist() == [x for row in rows for x in row]
        assert abs(plan.cost - oracle.sas_cost(M, J, r)) < 1e-9 * max(1.0, plan.cost)


U32 = 2.0 ** -24


def _accuracy(M, J, r):
    """(largest condition number, amplification, relative error bound) of the
    leaf systems at r, from the oracle's SVDs: amplification = max_v
    |V_v^{-1}|_2 max_v |D_v|_2, bound = amplification (2 + s)/2 u + u."""
    sv = oracle.leaf_singular_values(M, J, r)
    cond = max(v[0] / v[-1] for v, _ in sv)
    amp = max(1.0 / v[-1] for v, _ in sv) * max(d[0] for _, d in sv)
    return cond, amp, amp * (2 + len(r)) / 2 * U32 + U32


def test_leaf_accuracy_matches_oracle():
    """The planner's conditioning figures (FP64 power iteration on its own
    Gauss-Jordan inverse) against LAPACK SVDs of the oracle's leaf systems,
    on well- and ill-conditioned explicit pivot prefixes."""
    n_ill = 0
    for seed in range(40):
        rng = rng_for(1103, seed)
        M = int(rng.integers(6, 20))
        K, J = _subset(rng, M, int(rng.integers(2, min(M, 9) + 1)), rng.uniform(0.2, 0.9))
        r = list(K.levels[: int(rng.integers(0, len(K.levels) + 1))])
        level = (max(r) + 1) if r else 0
        mu = max(len(v) for v in oracle.level_nodes(M, J, level).values())
        if mu > 32:
            continue
        plan = native.SASPlan(M, J, pivots=r, host_only=True, weights_only=True)
        cond, amp, bound = _accuracy(M, J, r)
        n_ill += bound > native.SAS_MAX_REL_ERR
        if cond < 1e10:
            assert plan.leaf_cond == pytest.approx(cond, rel=1e-6), (seed, r)
            assert plan.amplification == pytest.approx(amp, rel=1e-6), (seed, r)
            assert plan.err_bound == pytest.approx(bound, rel=1e-6), (seed, r)
        else:  # numerically singular: both sides far above any accepted bound
            assert plan.err_bound > 1e3 * native.SAS_MAX_REL_ERR
    assert n_ill >= 3   # the set exercises refusals, not only good plans


def test_automatic_pivot_choice_minimises_lemma4_cost():
    """Among the prefixes of the pivots with mu* <= 32, 2^t <= 2^14 and a leaf
    error bound within the accuracy target, the planner takes the one of
    least Lemma 4 cost (the first such t on ties)."""
    for seed in range(40):
        rng = rng_for(1101, seed)
        M = int(rng.integers(8, 20))
        K, J = _subset(rng, M, int(rng.integers(3, min(M, 9) + 1)), rng.uniform(0.3, 0.9))
        P = oracle.pivots(M, J)
        best = None
        for t in range(0, min(len(P), 14) + 1):
            r = P[:t]
            level = (max(r) + 1) if r else 0
            mu = max(len(v) for v in oracle.level_nodes(M, J, level).values())
            if mu > 32 or _accuracy(M, J, r)[2] > native.SAS_MAX_REL_ERR:
                continue
            c = oracle.sas_cost(M, J, r)
            if best is None or c < best[0]:
                best = (c, r)
        plan = native.SASPlan(M, J, host_only=True)
        assert plan.pivots() == best[1]
        assert abs(plan.cost - best[0]) < 1e-9 * best[0]
        assert plan.err_bound <= native.SAS_MAX_REL_ERR


def test_ill_conditioned_plans_are_refused():
    """Explicit pivot prefixes whose leaf systems cannot meet the accuracy
    target are refused at creation, with the condition number in the message;
    the same r is accepted for the induced weights alone, and Lemma 4's
    automatic choice moves to a prefix that meets the bound.  Cases: an 80 %
    subset of a homogeneous set split at bits 0-3 and 9-13 at r = (0, 1, 2, 3)
    (nodes of up to 28 of 32 equispaced points: condition number 1.7e3), and
    26 consecutive integers at N = 2^16 with r = () (one node of 26 points
    within 2 pi 25 / 2^16 of each other: numerically singular)."""
    rng = rng_for(816, 0)
    K = homogeneous_support(14, 9, rng, levels=(0, 1, 2, 3, 9, 10, 11, 12, 13))
    keep = rng.random(len(K.J)) < 0.8
    sub = [int(j) for j, kp in zip(K.J, keep) if kp]
    for M, J, r in ((14, sub, [0, 1, 2, 3]), (16, list(range(26)), [])):
        with pytest.raises(native.HiDFTError) as ei:
            native.SASPlan(M, J, pivots=r, host_only=True)
        assert ei.value.status_name == "HIDFT_ERR_UNSUPPORTED"
        assert "condition number" in str(ei.value)
        w = native.SASPlan(M, J, pivots=r, host_only=True, weights_only=True)
        assert w.err_bound > native.SAS_MAX_REL_ERR and w.pivots() == r
        cond = _accuracy(M, J, r)[0]
        assert cond > 100
        if cond < 1e10:
            assert w.leaf_cond == pytest.approx(cond, rel=1e-6)
        auto = native.SASPlan(M, J, host_only=True)
        assert auto.err_bound <= native.SAS_MAX_REL_ERR and auto.pivots() != r


def test_homogeneous_support_reduces_to_the_plain_plan():
    rng = rng_for(1102, 0)
    sup = homogeneous_support(16, 8, rng)
    J = sup.J.tolist()
    plan = native.SASPlan(16, J, host_only=True)
    assert plan.pivots() == list(sup.levels) and plan.mu_max == 1
    assert plan.samples().tolist() == native.Plan(16, J, host_only=True).samples().tolist()


def test_rejects():
    J = [3, 17, 25, 27, 35]
    with pytest.raises(native.HiDFTError) as ei:
        native.SASPlan(6, J, pivots=[3], host_only=True)           # pivot 1 missing
    assert ei.value.status_name == "HIDFT_ERR_NOT_HOMOGENEOUS"
    with pytest.raises(native.HiDFTError) as ei:
        native.SASPlan(6, J, pivots=[3, 1], host_only=True)        # not ascending
    assert ei.value.status_name == "HIDFT_ERR_INVALID_ARGUMENT"
    with pytest.raises(native.HiDFTError) as ei:       # mu* = 64 > 32: no leaf solver
        native.SASPlan(10, list(range(64)), pivots=[], host_only=True)
    assert ei.value.status_name == "HIDFT_ERR_UNSUPPORTED"
    plan = native.SASPlan(10, list(range(64)), pivots=[], host_only=True, weights_only=True)
    assert plan.mu_max == 64 and plan.err_bound == float("inf")
    with pytest.raises(native.HiDFTError) as ei:       # refused before any device call
        plan.execute_ptr(8, 64, 8 + 4096, 64, 1, 8 + 8192)
    assert ei.value.status_name == "HIDFT_ERR_UNSUPPORTED"


@pytest.mark.parametrize("M", [3, 5, 8, 11, 14])
def test_powers_of_two_support(M):
    """J* = {1, 2, 4, ..., 2^{M-1}} (Sec. X).  Two elements 2^i > 2^j first
    meet at level j (2^i - 2^j = 2^j (2^{i-j} - 1), odd cofactor), so the
    pivots are {0, ..., M-2}: M - 1 splits separate the M elements (the
    paper writes {0, ..., M-1}; every internal level is a pivot).  J* is not
    homogeneous, and Shift-and-Sample with r = all pivots isolates each
    element (mu* = 1) only with 2^{M-1} = N/2 samples, far beyond the
    k^2 = M^2 work of the dense submatrix method, as the paper concludes."""
    J = [1 << i for i in range(M)]
    assert oracle.pivots(M, J) == list(range(M - 1))
    piv, hom = native.analyze(M, J)
    assert piv == list(range(M - 1)) and not hom
    plan = native.SASPlan(M, J, pivots=piv, host_only=True)
    assert plan.mu_max == 1
    assert plan.samples_per_signal == 1 << (M - 1)
    assert sorted(plan.samples().tolist()) == sorted(oracle.sample_pattern_recursive(M, piv))
