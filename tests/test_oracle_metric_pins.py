"""Pins of the oracle's error metrics, its index-set checks and Lemma 4's cost.

Every GPU parity assertion goes through ``oracle.rel_l2`` (and the reports
through ``oracle.max_abs``), so these are pinned on values worked out by hand:
a reduction over the wrong axis, a dropped square root or a constant return
fails here.  ``oracle.sas_cost`` is pinned on hand-counted nodes of small
supports (Sec. IX's worked example among them), where evaluating the nodes at
level r_max instead of r_max + 1 gives a different number.
"""
import math

import numpy as np
import pytest

import oracle


# ---------------------------------------------------------------------------
# rel_l2 and max_abs (per result: over the last axis)
# ---------------------------------------------------------------------------

def test_rel_l2_one_dimensional_hand_values():
    # ||[1,0] - [1,1]|| / ||[1,1]|| = 1 / sqrt(2)
    assert oracle.rel_l2(np.array([1, 0]), np.array([1, 1])) == pytest.approx(1 / math.sqrt(2),
                                                                              rel=1e-15)
    # complex: |i - 1| / |1| = sqrt(2)
    assert oracle.rel_l2(np.array([1j]), np.array([1.0])) == pytest.approx(math.sqrt(2), rel=1e-15)
    # error (3, 4i) against a reference of norm 10: 5 / 10
    ref = np.array([6.0, 8.0])
    assert oracle.rel_l2(ref + np.array([3.0, 4.0j]), ref) == pytest.approx(0.5, rel=1e-15)
    # no error: exactly zero
    assert oracle.rel_l2(ref, ref) == 0.0


def test_rel_l2_reduces_each_row_separately():
    # Three rows of length two (not square, so a reduction over the wrong
    # axis changes the shape): errors 1/5, 0 and 1 relative to their rows.
    ref = np.array([[3.0, 4.0], [1.0, 0.0], [0.0, 2.0j]])
    x = np.array([[3.0, 5.0], [1.0, 0.0], [0.0, 0.0]])
    got = oracle.rel_l2(x, ref)
    assert got.shape == (3,)
    np.testing.assert_allclose(got, [0.2, 0.0, 1.0], rtol=1e-15, atol=0)
    # rows scaled independently keep their own errors
    got2 = oracle.rel_l2(x * np.array([[10.0], [1.0], [1e-3]]), ref * np.array([[10.0], [1.0], [1e-3]]))
    np.testing.assert_allclose(got2, [0.2, 0.0, 1.0], rtol=1e-13, atol=0)


def test_rel_l2_is_a_norm_ratio_not_a_mean():
    # Two errors of 1 on a reference of norm 1 per entry...
    # ||(1, 1)|| / ||(1, 1)|| = 1, while a mean of |err| / |ref| per entry
    # would also be 1; an error concentrated in one entry separates them:
    # ||(2, 0)|| / ||(1, 1)|| = sqrt(2) (mean of ratios: 1).
    assert oracle.rel_l2(np.array([3.0, 1.0]), np.array([1.0, 1.0])) == pytest.approx(math.sqrt(2),
                                                                                     rel=1e-15)


def test_max_abs_hand_values():
    ref = np.array([[1.0, 2.0, 0.0], [0.0, 3.0, -1.0]])
    x = np.array([[1.0, 2.0 + 2.0j, 0.5], [0.0, 0.0, -1.0]])
    got = oracle.max_abs(x, ref)
    assert got.shape == (2,)
    np.testing.assert_allclose(got, [2.0, 3.0], rtol=0, atol=0)
    assert oracle.max_abs(np.array([1.0, 1.0 + 1.0j]), np.array([1.0, 0.0])) == pytest.approx(
        math.sqrt(2), rel=1e-15)
    assert oracle.max_abs(ref, ref).tolist() == [0.0, 0.0]


# ---------------------------------------------------------------------------
# Index-set checks of the problem statement (Sec. II: J is a subset of Z_N)
# ---------------------------------------------------------------------------

def test_check_index_set_rejects_out_of_range_and_duplicates():
    assert oracle.check_index_set(4, [0, 15, 7]) == [0, 15, 7]
    with pytest.raises(ValueError, match="outside"):
        oracle.check_index_set(4, [0, 16])
    with pytest.raises(ValueError, match="outside"):
        oracle.check_index_set(4, [-1, 3])
    with pytest.raises(ValueError, match="duplicate"):
        oracle.check_index_set(4, [3, 5, 3])
    # the checks guard every predicate that takes J
    with pytest.raises(ValueError):
        oracle.pivots(3, [1, 8])
    with pytest.raises(ValueError):
        oracle.is_homogeneous(3, [2, 2])


# ---------------------------------------------------------------------------
# Lemma 4: c1 s 2^s mu* + c2 sum_v mu(v)^2 over the nodes at level r_max + 1
# ---------------------------------------------------------------------------

def test_sas_cost_on_the_worked_example_of_sec_ix():
    # J = {0, 512, 1, 6, 7}, N = 2^10, r = (0, 1).  Nodes at level 2
    # (residues mod 4): {0, 512}, {1}, {6}, {7}; s = 2, mu* = 2.
    # 1.5 * 2 * 4 * 2 + 6 * (4 + 1 + 1 + 1) = 24 + 42 = 66.
    assert oracle.sas_cost(10, [0, 512, 1, 6, 7], [0, 1]) == 66.0


def test_sas_cost_on_hand_counted_supports():
    J = [3, 17, 25, 27, 35]  # N = 2^6, pivots {1, 3, 5}
    # r = (1): level 2, residues mod 4: {3, 27, 35} (3), {17, 25} (1).
    # 1.5 * 1 * 2 * 3 + 6 * (9 + 4) = 9 + 78 = 87.  (Level r_max = 1 would put
    # all five in one node: 15 + 150 = 165.)
    assert oracle.sas_cost(6, J, [1]) == 87.0
    # r = (1, 3): level 4, residues mod 16: {3, 35}, {17}, {25}, {27}.
    # 1.5 * 2 * 4 * 2 + 6 * (4 + 1 + 1 + 1) = 24 + 42 = 66.
    assert oracle.sas_cost(6, J, [1, 3]) == 66.0
    # r = (): one node at level 0 holding all of J: 6 * 25.
    assert oracle.sas_cost(6, J, []) == 150.0
    # r = all pivots (1, 3, 5): level 6, every element its own node.
    # 1.5 * 3 * 8 * 1 + 6 * 5 = 36 + 30 = 66.
    assert oracle.sas_cost(6, J, [1, 3, 5]) == 66.0


def test_positions_check_catches_permutations_and_phase_errors():
    """The per-row position check used at full size: exact coefficients pass
    in every row; a permutation of a row's outputs, or a phase error on each
    coefficient, fails in every row (each row's positions see it)."""
    from tests.positions import positions_vs_oracle
    from workloads import complex_normal, homogeneous_support, rng_for

    rng = rng_for(9101, 0)
    M, s, batch = 14, 8, 150
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    I = oracle.sample_set(M, J)
    c = complex_normal((batch, len(J)), rng)
    f = oracle.synthesize_samples(M, J, c, I).astype(np.complex64)
    exact = oracle.adjoint_coefficients(M, J, I, f.astype(np.complex128))
    ok = positions_vs_oracle(M, J, I, f, exact, 64, rng_for(9101, 1))
    assert ok.shape == (batch,) and ok.max() < 1e-12
    perm = exact[:, ::-1]
    assert positions_vs_oracle(M, J, I, f, perm, 64, rng_for(9101, 1)).min() > 0.1
    phase = exact * np.exp(1j * rng.uniform(0.01, 0.1, size=len(J)))
    assert positions_vs_oracle(M, J, I, f, phase, 64, rng_for(9101, 1)).min() > 1e-3
