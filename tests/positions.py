"""Element-wise oracle checks of every transform of a large batch.

At full size the oracle cannot afford every coefficient of every transform,
so each transform is compared with it on seeded positions of its own: rows go
in groups of `group` that share one draw of `n_pos` positions (one DFT
submatrix F(J_sel, I_r) per group, Lemma 1's adjoint form), and successive
groups draw afresh.  A permutation of outputs or a per-coefficient phase
error in any row shows up in its positions.
"""
import numpy as np

import oracle


def positions_vs_oracle(M, J, I, f_rows, got_rows, n_pos, rng, group=64):
    """Per-row rel-L2 of got_rows against the oracle on n_pos positions.

    f_rows: the samples exactly as the device read them (complex64 values),
    one row per transform; got_rows: the device's coefficients in J's order.
    Rows with k <= n_pos are compared on every position.
    """
    J = list(J)
    k = len(J)
    f_rows = np.asarray(f_rows).astype(np.complex64).astype(np.complex128)
    batch = f_rows.shape[0]
    errs = np.empty(batch)
    for lo in range(0, batch, group):
        hi = min(batch, lo + group)
        sel = np.arange(k) if k <= n_pos else np.sort(rng.choice(k, n_pos, replace=False))
        want = oracle.adjoint_coefficients(M, [J[t] for t in sel], I, f_rows[lo:hi], k=k)
        errs[lo:hi] = oracle.rel_l2(np.asarray(got_rows[lo:hi])[:, sel], want)
    return errs
