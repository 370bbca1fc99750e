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
        plan = native.SASPlan(M, J, pivots=r, host_only=True)
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


def test_automatic_pivot_choice_minimises_lemma4_cost():
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
            if mu > 32:
                continue
            c = oracle.sas_cost(M, J, r)
            if best is None or c < best[0]:
                best = (c, r)
        plan = native.SASPlan(M, J, host_only=True)
        assert plan.pivots() == best[1]
        assert abs(plan.cost - best[0]) < 1e-9 * best[0]


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
    plan = native.SASPlan(10, list(range(64)), pivots=[], host_only=True)   # mu* = 64
    assert plan.mu_max == 64
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
