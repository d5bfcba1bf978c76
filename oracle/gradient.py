"""Gradient of the sum of the k smallest fair eigenvalues (oracle side).

Unnormalized variant:

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

Normalized variant: the lambda_l are the eigenvalues of the pencil
(Z^T L Z, Z^T D Z) with Z a basis of null(F^T) (the problem of eq.
normal-prob-fair-1 with Theorem 2.1 applied to it), and h_l = Z y_l is
normalised by h_l^T D h_l = 1.  For a simple eigenvalue the derivative of a
generalized eigenvalue is y^T (dA - lambda dB) y, here
h^T dL h - lambda h^T dD h.  The weight w of edge {i, j} adds w to d_i and to
d_j, so h^T (dD/dw) h = h_i^2 + h_j^2, and
df/dw = sum_l [(h_il - h_jl)^2 - lambda_l (h_il^2 + h_jl^2)];
again each stored copy carries half.  A stored diagonal entry (i, i) adds w
to d_i only and leaves L unchanged: the half-per-copy formula then gives
-lambda_l h_il^2, which is its whole derivative, since it is stored once.

Neither derivation is in the paper; both follow from its Theorem 2.1 and
Proposition 3.3.  Pinned by finite differences of the dense oracle and by
automatic differentiation of a dense eigendecomposition (tests).
"""

from __future__ import annotations

import numpy as np

__all__ = ["eigsum_edge_gradient", "eigsum_edge_gradient_normalized"]


def eigsum_edge_gradient(rowptr, col, H):
    """Per stored entry (i, j): 0.5 * sum_l (H[i, l] - H[j, l])^2."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    H = np.asarray(H, dtype=np.float64)
    n = rowptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    diff = H[rows] - H[col]
    return 0.5 * np.einsum("ij,ij->i", diff, diff)


def eigsum_edge_gradient_normalized(rowptr, col, H, lam):
    """Per stored entry (i, j):
    0.5 * sum_l [(H[i, l] - H[j, l])^2 - lam[l] * (H[i, l]^2 + H[j, l]^2)],
    H D-orthonormal (H^T D H = I), lam the matching eigenvalues."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    H = np.asarray(H, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    if lam.size != H.shape[1]:
        raise ValueError("one eigenvalue per column of H")
    n = rowptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    diff = H[rows] - H[col]
    quad = (H * H) @ lam  # sum_l lam_l H[i, l]^2 per vertex
    return 0.5 * (np.einsum("ij,ij->i", diff, diff) - quad[rows] - quad[col])
