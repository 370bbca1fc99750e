"""CPU model of the split-precision arithmetic of group 1 on the matrix cores.

The first group of a transform (four or five stages of Lemma 3) is one fixed
unit-modulus matrix W per plan.  The matrix-core variants multiply each column
x of 16 or 32 samples by W with FP16 or BF16 operands and FP32 accumulation:

  FP16, two terms:   W = W1 + W2, x = x1 + x2 in FP16 after scaling the column by
                     a power of two that puts its largest component in
                     [2^14, 2^15); W x ~ W1 x1 + W1 x2 + W2 x1.
  BF16, three terms: W = W1 + W2 + W3, x = x1 + x2 + x3 in BF16, no scaling;
                     W x ~ W1 x1 + W1 x2 + W2 x1 + W1 x3 + W2 x2 + W3 x1.

This model rounds like the device (FP64 -> FP32 -> FP16 / BF16, round to
nearest even) and accumulates every product term in FP32, smallest first.  It
pins the precision the split arithmetic can reach, against the FP64 product
and against FP32 butterflies, independently of the HIP code.
"""
import numpy as np
import pytest

from workloads import rng_for


def _stage_matrix(rho, rng):
    """The product of rho radix-2 stages (stage u pairs bit rho-u; twiddle
    index (2^{u-1} - 1) + the bits above it), applied to the unit vectors in
    FP64, with random unit twiddles."""
    R = 1 << rho
    w = np.exp(-1j * np.pi * rng.random(R - 1) * 2.0)
    W = np.zeros((R, R), dtype=np.complex128)
    for c in range(R):
        x = np.zeros(R, dtype=np.complex128)
        x[c] = 1.0
        for u in range(1, rho + 1):
            b = rho - u
            for a in range(R):
                if (a >> b) & 1:
                    continue
                d = a | (1 << b)
                q = w[(1 << (u - 1)) - 1 + (a >> (b + 1))] * x[d]
                x[d] = x[a] - q
                x[a] = x[a] + q
        W[:, c] = x
    return W, w


def _bf16(x32):
    """FP32 -> BF16 (as FP32 values), round to nearest even."""
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return r.astype(np.uint32).view(np.float32)


def _f16(x32):
    return np.asarray(x32, dtype=np.float32).astype(np.float16).astype(np.float32)


def _real_blocks(W):
    """[Re W, -Im W; Im W, Re W], the real form of x -> W x."""
    return np.block([[W.real, -W.imag], [W.imag, W.real]])


def _columns(R, n, rng, spread=3.0):
    """n columns of R complex samples, CN(0, 1) times 10^U(-spread, spread)."""
    x = (rng.standard_normal((R, n)) + 1j * rng.standard_normal((R, n))) / np.sqrt(2)
    return x * 10.0 ** rng.uniform(-spread, spread, (1, n))


def _split_f16x2(W, x, scale=True):
    R = W.shape[0]
    A = _real_blocks(W)
    A32 = A.astype(np.float32)
    A1 = _f16(A32)
    A2 = _f16(A - A1.astype(np.float64))
    X = np.vstack([x.real, x.imag]).astype(np.float32)
    if scale:
        mx = np.max(np.abs(X), axis=0)
        e = (mx.view(np.uint32) >> 23) & 0xFF
        e = np.clip(e.astype(np.int64), 15, 254)
        sc = np.ldexp(np.float32(1.0), (141 - e).astype(np.int32)).astype(np.float32)
    else:
        sc = np.ones(X.shape[1], dtype=np.float32)
    Xs = (X * sc).astype(np.float32)
    X1 = _f16(Xs)
    X2 = _f16(Xs - X1)
    acc = np.zeros_like(Xs)
    for P, Q in ((A2, X1), (A1, X2), (A1, X1)):   # smallest first
        acc = (acc + (P.astype(np.float64) @ Q.astype(np.float64)).astype(np.float32)).astype(np.float32)
    Y = acc / sc
    return Y[:R].astype(np.float64) + 1j * Y[R:].astype(np.float64)


def _split_bf16x3(W, x):
    R = W.shape[0]
    A = _real_blocks(W)
    A1 = _bf16(A.astype(np.float32))
    r1 = A - A1.astype(np.float64)
    A2 = _bf16(r1.astype(np.float32))
    A3 = _bf16((r1 - A2.astype(np.float64)).astype(np.float32))
    X = np.vstack([x.real, x.imag]).astype(np.float32)
    X1 = _bf16(X)
    s1 = (X - X1).astype(np.float32)
    X2 = _bf16(s1)
    X3 = _bf16((s1 - X2).astype(np.float32))
    acc = np.zeros_like(X)
    for P, Q in ((A1, X3), (A2, X2), (A3, X1), (A1, X2), (A2, X1), (A1, X1)):
        acc = (acc + (P.astype(np.float64) @ Q.astype(np.float64)).astype(np.float32)).astype(np.float32)
    return acc[:R].astype(np.float64) + 1j * acc[R:].astype(np.float64)


def _butterflies_fp32(w, rho, x):
    """The same stages as FP32 butterflies (P + wQ by four FMAs' worth of
    FP32 operations, P - wQ = 2P - (P + wQ)), on every column."""
    R = 1 << rho
    w32 = w.astype(np.complex64)
    v = x.astype(np.complex64).copy()
    for u in range(1, rho + 1):
        b = rho - u
        for a in range(R):
            if (a >> b) & 1:
                continue
            d = a | (1 << b)
            t = w32[(1 << (u - 1)) - 1 + (a >> (b + 1))]
            s = (v[a] + t * v[d]).astype(np.complex64)
            v[d] = (np.complex64(2) * v[a] - s).astype(np.complex64)
            v[a] = s
    return v.astype(np.complex128)


def _rel(got, want):
    return np.linalg.norm(got - want, axis=0) / np.linalg.norm(want, axis=0)


@pytest.mark.parametrize("rho", [4, 5])
def test_split_precision_bounds(rho):
    """Both splits stay within a few FP32 roundings of the FP64 product, like
    FP32 butterflies, on columns spread over six decades."""
    rng = rng_for(9100, rho)
    W, w = _stage_matrix(rho, rng)
    x = _columns(1 << rho, 4000, rng)
    ref = W @ x
    e16 = _rel(_split_f16x2(W, x), ref)
    eb16 = _rel(_split_bf16x3(W, x), ref)
    e32 = _rel(_butterflies_fp32(w, rho, x), ref)
    print(f"radix {1 << rho}: FP16x2 max {e16.max():.2e}, BF16x3 max {eb16.max():.2e}, "
          f"FP32 butterflies max {e32.max():.2e}")
    assert e16.max() < 3e-7
    assert eb16.max() < 1.5e-7
    assert e32.max() < 3e-7
    # the three-term BF16 split is the more precise of the two
    assert np.median(eb16) < np.median(e16)


def test_f16_split_needs_the_column_scaling():
    """FP16's exponent range is narrow: without the per-column power-of-two
    scaling, columns of small magnitude lose their low bits (subnormals) and
    large ones overflow; with it, every column keeps the FP32 level."""
    rng = rng_for(9101, 0)
    W, _ = _stage_matrix(4, rng)
    x = _columns(16, 400, rng, spread=0.0)
    small, large = x * 1e-6, x * 1e5
    for cols in (small, large):
        ref = W @ cols
        assert _rel(_split_f16x2(W, cols), ref).max() < 3e-7
        with np.errstate(over="ignore", invalid="ignore"):
            unscaled = _split_f16x2(W, cols, scale=False)
        bad = ~np.isfinite(unscaled).all(axis=0) | (_rel(np.nan_to_num(unscaled), ref) > 1e-4)
        assert bad.all()


def test_stage_matrix_is_unitary_up_to_scale():
    """Every entry of W has modulus 1 and W W^H = R Id (each stage of
    butterflies with unit twiddles doubles the squared norm), so the outputs
    of a column have the magnitude of its inputs times at most sqrt(R): one
    power-of-two scale per column suffices."""
    for rho in (4, 5):
        W, _ = _stage_matrix(rho, rng_for(9102, rho))
        R = 1 << rho
        assert np.allclose(np.abs(W), 1.0, atol=1e-14)
        assert np.allclose(W @ W.conj().T, R * np.eye(R), atol=1e-12)
