"""Pins of the oracle's part-homogeneous and Shift-and-Sample functions."""
import numpy as np
import pytest

import oracle
from tests.golden import fixtures
from workloads import complex_normal, homogeneous_support, rng_for


@pytest.mark.parametrize("ex", fixtures.part_homogeneous_examples(),
                         ids=lambda e: f"{e['J']}-{e['r']}")
def test_printed_part_homogeneous_examples(ex):
    M, J, r = ex["M"], ex["J"], ex["r"]
    assert oracle.is_part_homogeneous(M, J, r), ex["cite"]
    nodes = oracle.level_nodes(M, J, ex["level"])
    got = sorted(sorted(J[t] for t in ts) for ts in nodes.values())
    assert got == ex["nodes"], ex["cite"]


def test_sas_example_sample_count():
    """Sec. IX: J = {0,512,1,6,7}, N = 1024 at level 2 needs mu* = 2 shifts of a
    4-point pattern: 8 samples, and they determine all five coefficients."""
    M, J, r = 10, [0, 512, 1, 6, 7], [0, 1]
    rows = oracle.sas_sample_set(M, r, 2)
    S = [x for row in rows for x in row]
    assert len(S) == 8
    c = complex_normal(5, rng_for(800, 0))
    f_S = oracle.synthesize_samples(M, J, c, S)
    assert oracle.rel_l2(oracle.solve_on_samples(M, J, S, f_S), c) < 1e-12


def test_hidft_values_are_induced_weights():
    """Eq. aliasing-homogeneous-tree (normalisation as in Sec. VII-B with the
    1/N of the inverse DFT restored): for r-part-homogeneous J and m in J,
    F(m, I_r) f_I = (2^s / N) mu_J(v(m), Ff), v(m) the node of m at level
    r_max + 1.  Checked by the dense product, for shifted samples too
    (Lemma 2: samples f(I_r + a) weight each c_l by exp(2 pi i a l / N))."""
    for seed in range(12):
        rng = rng_for(801, seed)
        M = int(rng.integers(6, 14))
        K = homogeneous_support(M, int(rng.integers(3, min(M, 7) + 1)), rng)
        # a random subset of a homogeneous set is part-homogeneous at the
        # first t pivots of the set
        keep = rng.random(len(K.J)) < 0.6
        J = [int(j) for j, kp in zip(K.J, keep) if kp] or [int(K.J[0])]
        t = int(rng.integers(0, len(K.levels) + 1))
        r = list(K.levels[:t])
        assert oracle.is_part_homogeneous(M, J, r)
        level = (max(r) + 1) if r else 0
        N, s = 1 << M, len(r)
        c = complex_normal(len(J), rng)
        I = sorted(oracle.sample_pattern_recursive(M, r))
        for a in (0, 1, 3):
            f_I = oracle.synthesize_samples(M, J, c, [(i + a) % N for i in I])
            hi = oracle.dft_submatrix(M, J, I) @ f_I
            w = c * np.exp(2j * np.pi * ((a * np.array(J, dtype=object)) % N).astype(np.float64) / N)
            mu = oracle.induced_weights(M, J, w, level)
            want = np.array([(2 ** s / N) * mu[j % (1 << level)] for j in J])
            assert np.max(np.abs(hi - want)) < 1e-10 * max(1.0, np.max(np.abs(want)))


def test_part_homogeneity_predicate():
    M, J = 6, [3, 17, 25, 27, 35]
    assert oracle.pivots(M, J) == [1, 3, 5]
    assert oracle.is_part_homogeneous(M, J, [1, 3])
    assert oracle.is_part_homogeneous(M, J, [1])
    assert not oracle.is_part_homogeneous(M, J, [3])        # pivot 1 missing
    assert oracle.is_part_homogeneous(M, J, [0, 1, 3])      # r may hold non-pivots
    assert oracle.is_part_homogeneous(M, J, [1, 3, 5])      # all pivots: homogeneous-like
    assert not oracle.is_part_homogeneous(M, J, [1, 5])     # pivot 3 below 5 missing


def test_sas_recovery_on_random_subsets():
    """Samples on the Shift-and-Sample pattern determine (Ff)_J: least squares
    on them recovers seeded coefficients (random subsets of homogeneous sets)."""
    for seed in range(10):
        rng = rng_for(802, seed)
        M = int(rng.integers(8, 14))
        K = homogeneous_support(M, int(rng.integers(4, 8)), rng)
        keep = rng.random(len(K.J)) < 0.5
        J = [int(j) for j, kp in zip(K.J, keep) if kp] or [int(K.J[0])]
        t = int(rng.integers(1, len(K.levels)))
        r = list(K.levels[:t])
        level = max(r) + 1
        mu = max(len(v) for v in oracle.level_nodes(M, J, level).values())
        S = [x for row in oracle.sas_sample_set(M, r, mu) for x in row]
        c = complex_normal(len(J), rng)
        f_S = oracle.synthesize_samples(M, J, c, S)
        assert oracle.rel_l2(oracle.solve_on_samples(M, J, S, f_S), c) < 1e-8
        assert oracle.sas_cost(M, J, r) > 0


def test_leaf_systems_two_element_node_closed_form():
    """A node of two elements l0, l1 (Sec. IX example: {0, 512} at N = 1024)
    has V = [[1, 1], [z0, z1]] with V^H V = [[2, 1 + conj(z0) z1], [., 2]], so
    its singular values are sqrt(2 +- 2 |cos(theta / 2)|), theta the angle
    between z0 and z1; the rows of D_v beyond the second add z^2, z^3, ..."""
    M, J, r = 10, [0, 512, 1, 6, 7], [0, 1]
    systems = oracle.leaf_systems(M, J, r)
    sv = oracle.leaf_singular_values(M, J, r)
    pair = [i for i, (V, D) in enumerate(systems) if V.shape[0] == 2]
    assert len(pair) == 1 and all(V.shape == (1, 1) for V, _ in
                                  (systems[i] for i in range(len(systems)) if i != pair[0]))
    # {0, 512}: theta = pi, the best-conditioned pair: both singular values sqrt(2)
    assert np.allclose(sv[pair[0]][0], [np.sqrt(2), np.sqrt(2)], atol=1e-12)
    for gap in (1, 3, 64, 100, 509):
        Jg = [5, 5 + 2 * gap]                     # one node at level 1 (r = (0,))
        theta = 2 * np.pi * 2 * gap / (1 << M)
        s_v = oracle.leaf_singular_values(M, Jg, [0])[0][0]
        c = abs(np.cos(theta / 2))
        assert np.allclose(s_v, [np.sqrt(2 + 2 * c), np.sqrt(2 - 2 * c)], rtol=1e-9), gap


def test_leaf_systems_equispaced_and_singleton_nodes():
    """A node that is a full coset of the top bits (l_t = l_0 + t N / mu) has
    V = diag(z_0^j) times the mu-point inverse-DFT matrix: all singular values
    sqrt(mu).  A single-element node has V = [1] and D = mu* unit numbers:
    singular value sqrt(mu*)."""
    M = 12
    for mu in (2, 4, 8, 32):
        step = (1 << M) // mu
        J = [7 + t * step for t in range(mu)] + [8]          # r = (0,): nodes {odd}, {8}
        sv = oracle.leaf_singular_values(M, J, [0])
        full = [x for x in sv if len(x[0]) == mu][0]
        single = [x for x in sv if len(x[0]) == 1][0]
        assert np.allclose(full[0], np.sqrt(mu), rtol=1e-12)
        assert np.allclose(full[1], np.sqrt(mu), rtol=1e-12)
        assert np.allclose(single[0], [1.0]) and np.allclose(single[1], [np.sqrt(mu)])


def test_leaf_systems_vandermonde_determinant():
    """|det V| = prod_{s < t} |z_t - z_s| (Vandermonde determinant), and the
    product of the singular values is |det V|: a textbook identity that fixes
    the node elements, their phases and the row powers of every leaf system."""
    for seed in range(6):
        rng = rng_for(803, seed)
        M = int(rng.integers(8, 16))
        K = homogeneous_support(M, int(rng.integers(4, 8)), rng)
        keep = rng.random(len(K.J)) < 0.7
        J = [int(j) for j, kp in zip(K.J, keep) if kp] or [int(K.J[0])]
        r = list(K.levels[: int(rng.integers(1, 3))])
        level = max(r) + 1
        nodes = list(oracle.level_nodes(M, J, level).values())
        sv = oracle.leaf_singular_values(M, J, r)
        for ts, (s_v, _) in zip(nodes, sv):
            z = [np.exp(2j * np.pi * J[t] / (1 << M)) for t in ts]
            det = 1.0
            for a in range(len(z)):
                for b in range(a):
                    det *= abs(z[a] - z[b])
            assert np.isclose(np.prod(s_v), det, rtol=1e-8, atol=1e-300), (seed, ts)
