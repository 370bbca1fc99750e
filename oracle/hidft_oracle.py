"""FP64 CPU oracle for the homogeneous-support DFT (arXiv 2211.15299).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product path
(the C-ABI library and its Python binding) never calls it, and this module
shares no code, tables or constants with the HIP path.

Everything here is written from the paper's definitions, slowly and plainly:

* index work (pivots, the homogeneity predicate, the pivoted sampling pattern,
  the plan orders and the butterfly twiddle exponents) follows the definitions
  of Sections VI-VIII with exact integer arithmetic;
* coefficients are obtained by the paper's simplest route of Section V-A (a dense solve):
  build the k x k submatrix F^{-1}(I, J) of the inverse DFT and solve the
  linear system f_I = F^{-1}(I, J) c by LU with partial pivoting, in complex128.
  For large k the algebraically identical adjoint form c = (N/k) F(J, I) f_I is
  used (Lemma 1 makes F(J, I_r) a scaled unitary matrix), see
  ``adjoint_coefficients``.

Conventions (Section II and Section IV): N = 2^M, omega = exp(-2 pi i / N),
(Ff)(m) = sum_n f(n) omega^{mn} (no normalisation) and
(F^{-1} c)(n) = (1/N) sum_m c(m) omega^{-mn}.

Readings of passages the text leaves garbled (each is also pinned by a test):

* The Hi-DFT identity F_J^0 f = |J| (Ff)_J drops the 1/N of the inverse DFT;
  with the paper's own DFT/IDFT conventions the correct statement is
  F(J, I_r) f_I = (k/N) (Ff)_J.  The factor 2 in the radix-2 split (Lemma 3) is
  likewise absent from the derivation in its proof.
* Algorithm 1 uses exp(+2 pi i a/N); the forward DFT sign of Lemma 3
  (omega_{r+1} = exp(-2 pi i / 2^{r+1})) is the one that reproduces (Ff)_J.
* Rows of the block factorisation of Corollary 2 are ordered by the recursion
  of the sampling pattern (I_r = I_{r-} followed by its translate); columns by
  q(j) = sum_u bit_{r_u}(j) 2^{u-1}.  The 4x4 matrix printed for
  J = {84, 305, 725, 992} reproduces entry for entry in this order.
"""
from __future__ import annotations

import math
from typing import Iterable, Sequence

import numpy as np
import scipy.linalg


# ---------------------------------------------------------------------------
# 2-adic index work (Section VI: congruence trees, pivots, homogeneity)
# ---------------------------------------------------------------------------

def nu2(x: int) -> int:
    """2-adic valuation of a nonzero integer (largest e with 2^e | x).

    Remark 1(1): the lowest common ancestor of two leaves of the congruence
    tree sits at level nu2(j_a - j_b).
    """
    x = int(x)
    if x == 0:
        raise ValueError("nu2 of zero is undefined")
    e = 0
    while x % 2 == 0:
        x //= 2
        e += 1
    return e


def check_index_set(M: int, J: Sequence[int]) -> list[int]:
    """Return J as a list of Python ints after the problem-statement checks:
    every index lies in Z_N (Section II) and indices are distinct."""
    N = 1 << M
    out = [int(j) for j in J]
    for j in out:
        if j < 0 or j >= N:
            raise ValueError(f"index {j} outside Z_N with N = 2^{M}")
    if len(set(out)) != len(out):
        raise ValueError("duplicate index in J")
    return out


def pivots(M: int, J: Sequence[int]) -> list[int]:
    """Pivot set P(J), sorted ascending, by brute force over all pairs.

    Remark 2 (pivot as gcd): level e is a pivot iff 2^e is the largest power of
    two dividing j_1 - j_2 for some j_1 != j_2 in J.  Differences are taken in
    Z_N (mod 2^M), which does not change nu2 for levels below M.
    """
    J = check_index_set(M, J)
    N = 1 << M
    arr = np.array(J, dtype=np.uint64)
    # O(k^2) pairs, one row at a time.  For a nonzero difference d the lowest
    # set bit d & -d equals 2^{nu2(d)}; OR-ing these powers of two over all
    # pairs leaves exactly the bits of the pivot levels.
    levels = 0
    with np.errstate(over="ignore"):
        for a in range(len(arr) - 1):
            d = (arr[a + 1:] - arr[a]) & np.uint64(N - 1)
            low = d & (~d + np.uint64(1))
            levels |= int(np.bitwise_or.reduce(low))
    return [e for e in range(M) if (levels >> e) & 1]


def is_power_of_two(k: int) -> bool:
    return k >= 1 and (k & (k - 1)) == 0


def is_homogeneous(M: int, J: Sequence[int]) -> bool:
    """Definition (homogeneous): T(J) has exactly log2 |J| pivots.

    Proposition 1 says there are always at least log2 |J| pivots, so this is the
    extreme case; it forces |J| to be a power of two.
    """
    J = check_index_set(M, J)
    k = len(J)
    if not is_power_of_two(k):
        return False
    return len(pivots(M, J)) == k.bit_length() - 1


def congruence_tree_levels(M: int, J: Sequence[int]) -> list[dict[int, list[int]]]:
    """The congruence tree T(J) level by level (Section VI).

    Level l holds the nonempty classes of J modulo 2^l, keyed by residue; the
    root (level 0) is J itself and the leaves (level M) are singletons.
    """
    J = check_index_set(M, J)
    levels = []
    for l in range(M + 1):
        nodes: dict[int, list[int]] = {}
        for j in J:
            nodes.setdefault(j % (1 << l), []).append(j)
        levels.append(nodes)
    return levels


def homogeneous_by_tree(M: int, J: Sequence[int]) -> bool:
    """Homogeneity through Proposition 2(2), checked on the explicit tree.

    Every split is into two children of equal weight, and if one node at a
    level splits, every node at that level splits.  Independent of ``pivots``.
    """
    levels = congruence_tree_levels(M, J)
    for l in range(M):
        splits = []
        for res, members in levels[l].items():
            children = [c for c in (res, res + (1 << l)) if c in levels[l + 1]]
            if len(children) == 2:
                w0 = len(levels[l + 1][children[0]])
                w1 = len(levels[l + 1][children[1]])
                if w0 != w1:
                    return False
                splits.append(True)
            else:
                splits.append(False)
        if any(splits) and not all(splits):
            return False
    return True


def pivots_by_tree(M: int, J: Sequence[int]) -> list[int]:
    """Pivots as levels of T(J) that hold a node with two children
    (Definition of pivots, Section VI)."""
    levels = congruence_tree_levels(M, J)
    out = []
    for l in range(M):
        if any(((res + (1 << l)) in levels[l + 1]) and (res in levels[l + 1])
               for res in levels[l]):
            out.append(l)
    return out


# ---------------------------------------------------------------------------
# Pivoted sampling pattern (Section VII, Definition of I_r)
# ---------------------------------------------------------------------------

def sample_pattern_recursive(M: int, r: Sequence[int]) -> list[int]:
    """I_r from its recursive definition, in recursion order.

    I_() = {0};  I_r = I_{r-} followed by I_{r-} translated by 2^{M-1-r_max}.
    The listing order (first the smaller pattern, then its translate) is the
    row order of the block factorisation of Corollary 2.
    """
    r = list(r)
    if r != sorted(r) or len(set(r)) != len(r):
        raise ValueError("pivot vector must be strictly ascending")
    if r and (r[0] < 0 or r[-1] >= M):
        raise ValueError("pivots must lie in [0, M)")
    pattern = [0]
    for u in range(len(r)):
        shift = 1 << (M - 1 - r[u])
        pattern = pattern + [x + shift for x in pattern]
    return pattern


def sample_pattern_closed_form(M: int, r: Sequence[int]) -> set[int]:
    """I_r from the non-recursive form: all sums of distinct 2^{M-1-r_u}."""
    s = len(r)
    out = set()
    for b in range(1 << s):
        out.add(sum((1 << (M - 1 - r[u])) for u in range(s) if (b >> u) & 1))
    return out


def sample_set(M: int, J: Sequence[int]) -> list[int]:
    """The k sample locations I_r for a homogeneous J, ascending."""
    if not is_homogeneous(M, J):
        raise ValueError("J is not homogeneous")
    return sorted(sample_pattern_recursive(M, pivots(M, J)))


# ---------------------------------------------------------------------------
# Plan orders and twiddle exponents (Lemma 3, Corollary 2, Algorithm 1)
# ---------------------------------------------------------------------------

def frequency_position(j: int, r: Sequence[int]) -> int:
    """q(j) = sum_u bit_{r_u}(j) 2^{u-1}: the column order of Corollary 2.

    The first half (q < k/2) is the left branch J_1 of the top split, the
    second half the right branch J_2; recursively inside each half.
    """
    return sum(((int(j) >> r[u]) & 1) << u for u in range(len(r)))


def frequency_positions(M: int, J: Sequence[int]) -> list[int]:
    """q(J[t]) for every t, in the caller's order of J."""
    r = pivots(M, J)
    return [frequency_position(j, r) for j in J]


def twiddle_exponents(M: int, J: Sequence[int]) -> list[tuple[int, int, int, int]]:
    """Butterfly twiddles of the radix-2 split, as exact integers.

    Lemma 3 combines the height-(n+1) Hi-DFT of f and of its translate by
    a = 2^{M-1-r} with the factor omega_{r+1}^{j} = exp(-2 pi i j / 2^{r+1})
    taken at the left descendant j (bit r of j is 0); the right descendant gets
    the negated factor.  Counting stages upward from the leaves (stage u uses
    pivot r_u), the butterflies of stage u are indexed by q_lo < 2^{u-1}, the
    frequency position of the node's low pivot bits, and the factor is
    exp(-i pi m / 2^{r_u}) with m = j mod 2^{r_u} for any j in J whose first
    u-1 pivot bits spell q_lo.

    Returns (u, q_lo, m, r_u) for u = 1..s and q_lo < 2^{u-1}, i.e. k-1 entries
    in the order stage-major, q_lo-minor.
    """
    J = check_index_set(M, J)
    r = pivots(M, J)
    s = len(r)
    if (1 << s) != len(J):
        raise ValueError("J is not homogeneous")
    by_q = {frequency_position(j, r): j for j in J}
    if len(by_q) != len(J):
        raise ValueError("q(j) is not a bijection: J is not homogeneous")
    out = []
    for u in range(1, s + 1):
        ru = r[u - 1]
        for q_lo in range(1 << (u - 1)):
            j = by_q[q_lo]
            out.append((u, q_lo, j % (1 << ru), ru))
    return out


# ---------------------------------------------------------------------------
# Fourier submatrices and the coefficient solve (Section V-A, Eq. submatrix)
# ---------------------------------------------------------------------------

def _phase_fraction(M: int, rows: Iterable[int], cols: Iterable[int]) -> np.ndarray:
    """((row * col) mod N) / N for every pair, with the product reduced exactly.

    uint64 products wrap modulo 2^64, and N = 2^M divides 2^64, so masking the
    wrapped product with N-1 gives the exact residue for every M <= 63.
    """
    N = 1 << M
    rows_a = np.array(list(rows), dtype=np.uint64)
    cols_a = np.array(list(cols), dtype=np.uint64)
    with np.errstate(over="ignore"):
        prod = (rows_a[:, None] * cols_a[None, :]) & np.uint64(N - 1)
    return prod.astype(np.float64) / float(N)


def dft_submatrix(M: int, rows: Sequence[int], cols: Sequence[int]) -> np.ndarray:
    """F(rows, cols) with entries exp(-2 pi i row col / N)   (Section II)."""
    return np.exp(-2j * np.pi * _phase_fraction(M, rows, cols))


def idft_submatrix(M: int, rows: Sequence[int], cols: Sequence[int]) -> np.ndarray:
    """F^{-1}(rows, cols) with entries (1/N) exp(+2 pi i row col / N) (Section IV)."""
    N = 1 << M
    return np.exp(2j * np.pi * _phase_fraction(M, rows, cols)) / N


def synthesize_samples(M: int, J: Sequence[int], c: np.ndarray,
                       I: Sequence[int], chunk: int = 2048) -> np.ndarray:
    """Samples f(i), i in I, of the signal in B^J whose DFT on J is c.

    f = F^{-1}(Z_N, J) (Ff)_J (Section V-A), evaluated only on the rows I.
    ``c`` may be (k,) or (batch, k); the result has the matching shape.  The
    matrix is formed ``chunk`` rows at a time to bound memory.
    """
    I = list(I)
    c = np.asarray(c, dtype=np.complex128)
    cm = c[None, :] if c.ndim == 1 else c
    out = np.empty((cm.shape[0], len(I)), dtype=np.complex128)
    for lo in range(0, len(I), chunk):
        A = idft_submatrix(M, I[lo:lo + chunk], J)
        out[:, lo:lo + chunk] = cm @ A.T
    return out[0] if c.ndim == 1 else out


def synthesize_samples_fft(M: int, J: Sequence[int], c: np.ndarray,
                           I: Sequence[int]) -> np.ndarray:
    """The same samples as synthesize_samples, through the full-length
    inverse DFT: the spectrum that is c on J and zero elsewhere, transformed
    by numpy.fft.ifft (which includes the 1/N of F^{-1}, Section II) and read
    at I.  O(N log N) per signal instead of O(k |I|): for large k at moderate
    N (one N-point complex128 vector per signal).
    """
    J = np.asarray(list(J), dtype=np.int64)
    I = np.asarray(list(I), dtype=np.int64)
    N = 1 << M
    if len(np.unique(J)) != len(J) or (len(J) and (J.min() < 0 or J.max() >= N)):
        raise ValueError("J must be distinct indices in [0, N)")
    c = np.asarray(c, dtype=np.complex128)
    cm = c[None, :] if c.ndim == 1 else c
    out = np.empty((cm.shape[0], len(I)), dtype=np.complex128)
    spec = np.zeros(N, dtype=np.complex128)
    for b in range(cm.shape[0]):
        spec[:] = 0
        spec[J] = cm[b]
        out[b] = np.fft.ifft(spec)[I]
    return out[0] if c.ndim == 1 else out


def solve_coefficients(M: int, J: Sequence[int], I: Sequence[int],
                       f_I: np.ndarray) -> np.ndarray:
    """(Ff)_J from k samples by solving f_I = F^{-1}(I, J) (Ff)_J.

    This is the paper's trivial O(k^2)-per-signal route (Eq. submatrix-method),
    done with a dense LU factorisation with partial pivoting (LAPACK zgetrf /
    zgetrs) in complex128.  ``f_I`` may be (k,) or (batch, k).
    """
    A = idft_submatrix(M, I, J)
    f_I = np.asarray(f_I, dtype=np.complex128)
    lu = scipy.linalg.lu_factor(A, check_finite=True)
    if f_I.ndim == 1:
        return scipy.linalg.lu_solve(lu, f_I)
    return scipy.linalg.lu_solve(lu, f_I.T).T


def adjoint_coefficients(M: int, J: Sequence[int], I: Sequence[int],
                         f_I: np.ndarray, k: int | None = None,
                         chunk: int = 2048) -> np.ndarray:
    """(Ff)_J = (N/k) F(J, I) f_I for a homogeneous J sampled on I = I_r.

    Lemma 1 shows the aliasing pattern of I_r vanishes on every difference of
    two distinct elements of J, so F(J, I_r) F(J, I_r)^H = k Id and the inverse
    of F^{-1}(I_r, J) is (N/k) F(J, I_r): the same answer as the LU solve,
    without a factorisation.  Valid only for I = I_r of a homogeneous J.

    ``J`` may be any subset of the support (then pass the support size ``k``)
    to evaluate selected coefficients only.  ``f_I`` may be (k,) or (batch, k).
    The matrix is formed ``chunk`` rows at a time to bound memory.
    """
    N = 1 << M
    J = list(J)
    k = len(J) if k is None else k
    f_I = np.asarray(f_I, dtype=np.complex128)
    fm = f_I[None, :] if f_I.ndim == 1 else f_I
    out = np.empty((fm.shape[0], len(J)), dtype=np.complex128)
    for lo in range(0, len(J), chunk):
        F = dft_submatrix(M, J[lo:lo + chunk], I)
        out[:, lo:lo + chunk] = fm @ F.T
    out *= N / k
    return out[0] if f_I.ndim == 1 else out


def coefficient_at(M: int, j: int, I: Sequence[int], f_I: np.ndarray, k: int) -> complex:
    """One coefficient (Ff)(j) = (N/k) sum_{i in I_r} f(i) omega^{ij}.

    The one-row form of ``adjoint_coefficients``, for spot checks of large
    transforms one output at a time.
    """
    N = 1 << M
    row = dft_submatrix(M, [j], I)[0]
    return complex((N / k) * np.dot(row, np.asarray(f_I, dtype=np.complex128)))


def coefficients(M: int, J: Sequence[int], f_I: np.ndarray, method: str = "auto") -> np.ndarray:
    """(Ff)_J for a homogeneous J from samples on I_r (ascending order).

    method: "lu" (dense solve), "adjoint", or "auto" (LU up to k = 4096).
    """
    I = sample_set(M, J)
    if method == "auto":
        method = "lu" if len(J) <= 4096 else "adjoint"
    if method == "lu":
        return solve_coefficients(M, J, I, f_I)
    if method == "adjoint":
        return adjoint_coefficients(M, J, I, f_I)
    raise ValueError(method)


# ---------------------------------------------------------------------------
# Error report (per result)
# ---------------------------------------------------------------------------

def rel_l2(x: np.ndarray, ref: np.ndarray) -> float:
    """||x - ref||_2 / ||ref||_2 over the last axis (a float for 1-D input)."""
    x = np.asarray(x, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    num = np.linalg.norm(x - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return num / den


def max_abs(x: np.ndarray, ref: np.ndarray) -> float:
    return np.max(np.abs(np.asarray(x) - np.asarray(ref)), axis=-1)


def op_count(k: int) -> int:
    """Theorem 1: 1.5 A log2 A + A arithmetic operations for A = k samples."""
    s = k.bit_length() - 1
    return int(1.5 * k * s + k) if k > 1 else 1


# ---------------------------------------------------------------------------
# Part-homogeneous supports, induced weights and Shift-and-Sample (Sec. VI,
# Sec. VII-B, Sec. IX, Algorithm 2)
# ---------------------------------------------------------------------------

def level_nodes(M: int, J: Sequence[int], level: int) -> dict[int, list[int]]:
    """Nodes of T(J) at `level`: positions t of J grouped by J[t] mod 2^level.

    Keys are the residues, values the caller positions t in ascending order.
    """
    J = check_index_set(M, J)
    nodes: dict[int, list[int]] = {}
    for t, j in enumerate(J):
        nodes.setdefault(j % (1 << level), []).append(t)
    return nodes


def is_part_homogeneous(M: int, J: Sequence[int], r: Sequence[int]) -> bool:
    """Def. part-homogeneous: J has no pivot at a level <= r_max outside r."""
    r = list(r)
    if not r:
        return True
    return all(p in r for p in pivots(M, J) if p <= max(r))


def induced_weights(M: int, J: Sequence[int], w: np.ndarray, level: int) -> dict[int, complex]:
    """mu_J(v, w) = sum of w over the elements of each node v at `level`
    (Sec. VI, induced weight), keyed by the node's residue mod 2^level."""
    w = np.asarray(w, dtype=np.complex128)
    return {res: complex(np.sum(w[ts])) for res, ts in level_nodes(M, J, level).items()}


def sas_sample_set(M: int, r: Sequence[int], shifts: int) -> list[list[int]]:
    """Rows j = 0..shifts-1 of the Shift-and-Sample pattern: I_r + j (mod N),
    each row in ascending order of I_r (Algorithm 2, step 3)."""
    N = 1 << M
    base = sorted(sample_pattern_recursive(M, r))
    return [[(i + j) % N for i in base] for j in range(shifts)]


def sas_cost(M: int, J: Sequence[int], r: Sequence[int]) -> float:
    """Lemma 4: c1 s 2^s mu* + c2 sum_v mu(v)^2 with c1 = 3/2, c2 = 6, the
    nodes v taken at level r_max + 1 (level 0 when r is empty)."""
    s = len(r)
    level = (max(r) + 1) if s else 0
    mus = [len(v) for v in level_nodes(M, J, level).values()]
    return 1.5 * s * (1 << s) * max(mus) + 6.0 * sum(m * m for m in mus)


def solve_on_samples(M: int, J: Sequence[int], S: Sequence[int], f_S: np.ndarray) -> np.ndarray:
    """(Ff)_J from samples f(S), |S| >= |J|: the least-squares solution of
    f_S = F^{-1}(S, J) (Ff)_J (Eq. submatrix-method with more rows than
    unknowns; exact for f in B^J when F^{-1}(S, J) has full column rank)."""
    A = idft_submatrix(M, S, J)
    f_S = np.asarray(f_S, dtype=np.complex128)
    sol, *_ = np.linalg.lstsq(A, f_S.T if f_S.ndim == 2 else f_S, rcond=None)
    return sol.T if f_S.ndim == 2 else sol


def leaf_systems(M: int, J: Sequence[int], r: Sequence[int]) -> list[tuple[np.ndarray, np.ndarray]]:
    """The leaf systems of Shift-and-Sample at r (Algorithm 2, Eq. alg1_system),
    one per node v at level r_max + 1: (V_v, D_v), where D_v[j][t] = z_t^j for
    the mu* shifts j and z_t = exp(2 pi i l_t / N) for the node's elements l_t
    (exact integer phase j l_t mod N), and V_v its first mu(v) rows, the square
    system the solve inverts."""
    J = check_index_set(M, J)
    level = (max(r) + 1) if len(r) else 0
    nodes = list(level_nodes(M, J, level).values())
    mu_star = max(len(ts) for ts in nodes)
    out = []
    for ts in nodes:
        D = np.exp(2j * np.pi * _phase_fraction(M, range(mu_star), [J[t] for t in ts]))
        out.append((D[: len(ts)], D))
    return out


def leaf_singular_values(M: int, J: Sequence[int], r: Sequence[int]) -> list[tuple[np.ndarray, np.ndarray]]:
    """Singular values (LAPACK SVD, descending) of each node's V_v and D_v."""
    return [(np.linalg.svd(V, compute_uv=False), np.linalg.svd(D, compute_uv=False))
            for V, D in leaf_systems(M, J, r)]
