"""Fair spectral embedding with a general constraint matrix F (oracle; test
infrastructure).

The paper builds F from disjoint group labels (Lemma 2.1), but nothing in
the method after that uses the structure of F: the nullspace basis
(Section 3.1), the projector P = I - C (C^T C)^{-1} C^T with C = D^{-1/2} F
(Section 3.2, eq. mv-Pw) and the deflated operator (eq. asigma) are defined
for any n x m matrix F.  Two uses of that generality appear in the paper:
the random-Laplacian workload, whose F is a random placeholder
(Section 5, "Random Laplacian"), and overlapping groups, where F may lose
rank and a rank-revealing factorization comes first (Section 6).

Rank: range(F) is taken to be spanned by the left singular vectors whose
singular value exceeds rank_tol times the largest (SVD as one library
step).  Then r = rank(F) directions are constrained and the fair problem
lives on an (n - r)-dimensional subspace.  For the normalized variant the
rank is read from C = D^{-1/2} F in the implicit tier and the operator, and
from F in the dense tier; D is positive definite, so both have the same
exact rank.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .fairsc import _ImplicitNullspace, _as_csr, _operator_matrix, degrees, laplacian

__all__ = [
    "membership_fairness_matrix",
    "general_constraint_matrix",
    "range_basis",
    "fair_eigs_dense_general",
    "fair_eigs_implicit_general",
    "apply_deflated_operator_general",
]


def membership_fairness_matrix(G) -> np.ndarray:
    """F_0 = G - 1 z^T with z = G^T 1 / n for a 0/1 membership matrix G
    (n x g; a row may hold several ones).

    For disjoint groups this is Lemma 2.1's F_0, whose columns sum to zero,
    so one of them is dependent and the lemma keeps h - 1.  With overlapping
    memberships no fixed column can be dropped, so all are kept and the rank
    is revealed numerically (Section 6)."""
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    z = G.sum(axis=0) / n
    return G - np.ones((n, 1)) * z[None, :]


def general_constraint_matrix(W, F, normalized) -> np.ndarray:
    """C = D^{-1/2} F (normalized, Section 3.2) or C = F."""
    F = np.asarray(F, dtype=np.float64)
    if normalized:
        return F / np.sqrt(degrees(W))[:, None]
    return F.copy()


def range_basis(A, rank_tol=1e-6):
    """(U_r, r): orthonormal basis of the numerical range of A (thin SVD,
    singular values above rank_tol * the largest)."""
    A = np.asarray(A, dtype=np.float64)
    if A.shape[1] == 0:
        return np.zeros((A.shape[0], 0)), 0
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    r = int(np.sum(s > rank_tol * s[0])) if s[0] > 0 else 0
    return U[:, :r], r


def fair_eigs_dense_general(W, F, k, normalized, rank_tol=1e-6):
    """Tier A with a general F: Z = orthonormal basis of null(F^T) from a
    full SVD of F (the columns of U beyond the numerical rank r), then the
    (generalized) symmetric eigenproblem on Z^T L Z (Z^T D Z) as for group
    constraints.  Returns (lam[k] ascending, H n x k, r), F^T H = 0 and
    H^T D H = I (normalized) or H^T H = I."""
    W = _as_csr(W)
    n = W.shape[0]
    F = np.asarray(F, dtype=np.float64).reshape(n, -1)
    L = laplacian(W).toarray()
    if F.shape[1]:
        U, s, _ = np.linalg.svd(F, full_matrices=True)
        r = int(np.sum(s > rank_tol * s[0])) if s.size and s[0] > 0 else 0
    else:
        U, r = np.eye(n), 0
    if not 1 <= k <= n - r:
        raise ValueError("k out of range")
    Z = U[:, r:]
    M = Z.T @ L @ Z
    M = 0.5 * (M + M.T)
    if normalized:
        d = degrees(W)
        B = Z.T @ (d[:, None] * Z)
        lam, Y = sla.eigh(M, 0.5 * (B + B.T))
    else:
        lam, Y = np.linalg.eigh(M)
    return lam[:k].copy(), Z @ Y[:, :k], r


def fair_eigs_implicit_general(W, F, k, normalized, rank_tol=1e-6, tol=1e-12, seed=0, ncv=None):
    """Tier B with a general F: the nullspace of C^T held as Householder
    reflectors of a QR of U_r (the range basis of C), and ARPACK ("SA") on
    y -> V^T L_n V y (FairSC variant 1, eq. lveig).  No n x n matrix is
    formed.  Returns (lam[k], H n x k, r)."""
    W = _as_csr(W)
    n = W.shape[0]
    A = _operator_matrix(W, normalized)
    Ur, r = range_basis(general_constraint_matrix(W, F, normalized), rank_tol)
    if r:
        ns = _ImplicitNullspace(Ur)

        def mv(y):
            return ns.VT(A @ ns.V(y)).ravel()

        back = ns.V
    else:

        def mv(y):
            return A @ np.asarray(y).ravel()

        def back(y):
            return np.asarray(y).reshape(n, -1)

    dim = n - r
    op = spla.LinearOperator((dim, dim), matvec=mv, dtype=np.float64)
    rng = np.random.Generator(np.random.Philox(int(seed)))
    if ncv is None:
        ncv = min(dim, max(2 * k + 1, 4 * k, 40))
    lam, Y = spla.eigsh(op, k=k, which="SA", tol=tol, v0=rng.standard_normal(dim), ncv=ncv)
    order = np.argsort(lam)
    X = back(Y[:, order])
    if normalized:
        X = X / np.sqrt(degrees(W))[:, None]
    return lam[order], X, r


def apply_deflated_operator_general(W, F, normalized, sigma, X, rank_tol=1e-6):
    """Y = L^sigma X = P(L_n (P X)) - sigma P X + sigma X (eq. asigma, the
    matvec of Section 3.4) with P w = w - C z and z the minimum-norm
    least-squares solution of C z = w (eq. mv-Pw; singular values of C below
    rank_tol times the largest are treated as zero)."""
    W = _as_csr(W)
    A = _operator_matrix(W, normalized)
    C = general_constraint_matrix(W, F, normalized)
    X = np.asarray(X, dtype=np.float64)
    X2 = X.reshape(X.shape[0], -1)

    def P(w):
        if C.shape[1] == 0:
            return w
        z = np.linalg.lstsq(C, w, rcond=rank_tol)[0]
        return w - C @ z

    Xp = P(X2)
    Y = P(A @ Xp) - sigma * Xp + sigma * X2
    return Y.reshape(X.shape)
