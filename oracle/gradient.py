"""Gradient of the sum of the k smallest fair eigenvalues (oracle side).

For the unnormalized variant, f(W) = sum_{i<=k} lambda_i = the minimum of
tr(X^T L(W) X) over X^T X = I, F^T X = 0 (Theorem 2.1 applied to the
restricted operator of Proposition 3.3).  F depends only on the groups, so
when lambda_k < lambda_{k+1} the minimiser X is locally unique up to rotation
and the envelope (Hellmann-Feynman) argument gives
df/dw_e = tr(X^T (dL/dw_e) X).  An undirected edge {i, j} of weight w enters
L as w (e_i - e_j)(e_i - e_j)^T, so df/dw_e = ||X_i - X_j||^2.  Each of the two
stored copies (i, j) and (j, i) carries half of it, so that the inner product
of the gradient with any symmetric perturbation of the stored values is the
directional derivative.  The shift sigma is treated as a constant.

This derivation is not in the paper; it follows from its Theorem 2.1 and
Proposition 3.3.  Pinned by finite differences of the dense oracle and by
automatic differentiation of a dense eigendecomposition (tests).
"""

from __future__ import annotations

import numpy as np

__all__ = ["eigsum_edge_gradient"]


def eigsum_edge_gradient(rowptr, col, H):
    """Per stored entry (i, j): 0.5 * sum_l (H[i, l] - H[j, l])^2."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    H = np.asarray(H, dtype=np.float64)
    n = rowptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    diff = H[rows] - H[col]
    return 0.5 * np.einsum("ij,ij->i", diff, diff)
