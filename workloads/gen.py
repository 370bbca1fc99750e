"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws inputs only.  It computes nothing that the transform computes:
no pivots are detected, no sample sets, orders or twiddles are derived, and no
coefficients or samples are obtained from one another.  Both the HIP path and
the FP64 oracle receive what these functions return.

Homogeneous supports.  By Proposition 2(2) a set J subset of Z_N is homogeneous
iff its congruence tree splits every node, into equal halves, at each of s
levels (the pivots) and splits no node elsewhere.  Equivalently: bit l of j is
free at a pivot level l, and at every other level it is a fixed function of
the bits of j at the pivot levels below l.  ``homogeneous_support`` draws such
a set directly from that description, then applies an odd dilation and a
translation modulo N (both keep every 2-adic valuation of a difference, hence
the pivots).  Every homogeneous set arises this way.

Seeds follow numpy.random.SeedSequence([221115299, config_id, instance_id]).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PAPER_SEED = 221115299


def rng_for(config_id: int, instance_id: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([PAPER_SEED, int(config_id), int(instance_id)])))


@dataclass
class Support:
    M: int                 # N = 2^M
    J: np.ndarray          # uint64[k], in the (shuffled) caller order
    levels: tuple          # the split levels the set was built with, ascending

    @property
    def N(self) -> int:
        return 1 << self.M

    @property
    def k(self) -> int:
        return len(self.J)


def _affine(M: int, x: np.ndarray, rng: np.random.Generator, dilate: bool,
            translate: bool) -> np.ndarray:
    N = 1 << M
    mask = np.uint64(N - 1)
    d = int(rng.integers(0, N // 2)) * 2 + 1 if (dilate and M > 0) else 1
    t = int(rng.integers(0, N)) if (translate and M > 0) else 0
    with np.errstate(over="ignore"):
        return (x.astype(np.uint64) * np.uint64(d) + np.uint64(t)) & mask


def homogeneous_support(M: int, s: int, rng: np.random.Generator, *,
                        levels=None, dilate: bool = True, translate: bool = True,
                        shuffle: bool = True) -> Support:
    """A seeded homogeneous J subset of Z_{2^M} with |J| = 2^s.

    levels: the s split levels (drawn uniformly from {0..M-1} when None).
    Non-split bits are independent uniformly random Boolean functions of the
    split bits below them.
    """
    if not (0 <= s <= M <= 63):
        raise ValueError("need 0 <= s <= M <= 63")
    if levels is None:
        levels = sorted(rng.choice(M, size=s, replace=False).tolist()) if s else []
    levels = tuple(int(x) for x in sorted(levels))
    if len(levels) != s or len(set(levels)) != s or (s and (levels[0] < 0 or levels[-1] >= M)):
        raise ValueError("bad levels")
    k = 1 << s
    b = np.arange(k, dtype=np.uint64)          # b's bit u is the bit at levels[u]
    x = np.zeros(k, dtype=np.uint64)
    n_below = 0
    for l in range(M):
        if n_below < s and levels[n_below] == l:
            bit = (b >> np.uint64(n_below)) & np.uint64(1)
            n_below += 1
        else:
            # a random Boolean function of the n_below split bits under level l
            table = rng.integers(0, 2, size=1 << n_below, dtype=np.uint64)
            bit = table[(b & np.uint64((1 << n_below) - 1)).astype(np.int64)]
        x |= bit << np.uint64(l)
    J = _affine(M, x, rng, dilate, translate)
    if shuffle:
        J = J[rng.permutation(k)]
    return Support(M, J, levels)


def elementary_support(M: int, s: int, rng: np.random.Generator, *,
                       shuffle: bool = False) -> Support:
    """{(d x + t) mod N : x < 2^s} with a seeded odd d and t in [0, N)."""
    x = np.arange(1 << s, dtype=np.uint64)
    J = _affine(M, x, rng, True, True)
    if shuffle:
        J = J[rng.permutation(len(J))]
    return Support(M, J, tuple(range(s)))


def composite_support(M: int, blocks: list, rng: np.random.Generator) -> Support:
    """Direct sum A + 2^{t} B + ... of homogeneous blocks on disjoint bit ranges.

    blocks: list of (lo, width, s) -- a homogeneous set of 2^s elements of
    Z_{2^width} placed at bits [lo, lo + width).  Ranges must be disjoint.
    The split levels of the sum are the union of the blocks' shifted levels.
    """
    used = set()
    J = np.zeros(1, dtype=np.uint64)
    levels = []
    for lo, width, s in blocks:
        rng_bits = set(range(lo, lo + width))
        if rng_bits & used or lo + width > M:
            raise ValueError("blocks overlap or exceed M")
        used |= rng_bits
        blk = homogeneous_support(width, s, rng, shuffle=False)
        levels += [lo + l for l in blk.levels]
        J = (J[:, None] + (blk.J.astype(np.uint64)[None, :] << np.uint64(lo))).reshape(-1)
    J = J[rng.permutation(len(J))]
    return Support(M, J, tuple(sorted(levels)))


def uneven_instances(n: int, config_id: int = 3, composites: int = 64) -> list:
    """The uneven batch: n instances, each (M, Support) with its own seeded J.

    Instance i draws from rng_for(config_id, i).  The first `composites` are
    direct sums of two or three homogeneous blocks on disjoint bit ranges
    (M uniform on 14..24, block widths 3..6 bits, gaps of 0..2 bits); the
    others are homogeneous with N = 2^M, M uniform on 12..24, and k = 2^s, s
    uniform on 6..min(14, M - 2) (so k <= N/4).
    """
    out = []
    for i in range(n):
        rng = rng_for(config_id, i)
        if i < composites:
            M = int(rng.integers(14, 25))
            widths = [int(rng.integers(3, 7)) for _ in range(3)]
            blocks, lo = [], 0
            for w in widths:
                if lo + w > M:
                    break
                blocks.append((lo, w, int(rng.integers(1, w))))
                lo += w + int(rng.integers(0, 3))
            sup = composite_support(M, blocks, rng)
        else:
            M = int(rng.integers(12, 25))
            s = int(rng.integers(6, min(14, M - 2) + 1))
            sup = homogeneous_support(M, s, rng)
        out.append((M, sup))
    return out


def gap_support(M: int, sizes, rng: np.random.Generator, *, max_tries: int = 1000,
                shuffle: bool = True) -> Support:
    """A proper generalized arithmetic progression of dimension d = len(sizes)
    (Sec. IX-B, Def. GAP): {a + n_1 s_1 + ... + n_d s_d mod N : 0 <= n_i < N_i},
    with the offset a and the common differences s_i drawn uniformly from Z_N
    (odd or even), redrawn until all prod(N_i) sums are distinct (proper).

    GAPs are not built from split levels: ``levels`` is empty.
    """
    sizes = [int(n) for n in sizes]
    N = 1 << M
    k = int(np.prod(sizes)) if sizes else 1
    if k > N:
        raise ValueError("a proper GAP has at most N elements")
    grids = np.meshgrid(*[np.arange(n, dtype=np.int64) for n in sizes], indexing="ij")
    for _ in range(max_tries):
        a = int(rng.integers(0, N))
        steps = [int(x) for x in rng.integers(1, N, size=len(sizes))]
        J = np.full(grids[0].shape if sizes else (), a, dtype=np.int64)
        for g, st in zip(grids, steps):
            J = J + g * st
        J = (J.reshape(-1) % N).astype(np.uint64)
        if len(np.unique(J)) == k:
            if shuffle:
                J = J[rng.permutation(k)]
            return Support(M, J, ())
    raise RuntimeError("no proper GAP found; use smaller sizes or a larger N")


def arithmetic_progression(M: int, k: int, rng: np.random.Generator, alpha: int,
                           shuffle: bool = True) -> Support:
    """{a + i s mod N : i < k} with common difference s = 2^alpha * (odd), a
    and the odd factor drawn uniformly (Sec. IX-A, arithmetic progressions of
    arbitrary common difference).  Needs k <= 2^(M - alpha) (distinct terms)."""
    N = 1 << M
    if alpha < 0 or alpha >= M or k > (N >> alpha):
        raise ValueError("need 0 <= alpha < M and k <= 2^(M - alpha)")
    a = int(rng.integers(0, N))
    odd = int(rng.integers(0, max(N >> (alpha + 1), 1))) * 2 + 1
    s = (odd << alpha) % N
    J = ((a + np.arange(k, dtype=np.int64) * s) % N).astype(np.uint64)
    if shuffle:
        J = J[rng.permutation(k)]
    return Support(M, J, ())


def complex_normal(shape, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    """Circular standard complex normal CN(0, scale^2): Re, Im ~ N(0, scale^2/2)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * (scale / np.sqrt(2.0))


def log_uniform_coefficients(shape, rng: np.random.Generator, lo: float = 1e-3,
                             hi: float = 1e3) -> np.ndarray:
    """Magnitudes log-uniform on [lo, hi], phases uniform on [0, 2 pi)."""
    mag = np.exp(rng.uniform(np.log(lo), np.log(hi), size=shape))
    ph = rng.uniform(0.0, 2.0 * np.pi, size=shape)
    return mag * np.exp(1j * ph)


def sample_values(M: int, k: int, batch: int, rng: np.random.Generator,
                  dtype=np.complex64) -> np.ndarray:
    """Random sample values for `batch` signals, shape (batch, k).

    Draws i.i.d. CN(0, k / N^2) values: the distribution of the k samples of a
    signal whose k DFT coefficients are i.i.d. CN(0, 1) (the sampling matrix is
    a scaled unitary matrix, so the draw is identical in law).  Used where only
    the shape and scale of realistic inputs matter (timing); parity cases
    compare against the oracle on whatever samples were drawn.
    """
    N = float(1 << M)
    return complex_normal((batch, k), rng, scale=np.sqrt(k) / N).astype(dtype)
