"""Fair spectral embedding, restated plainly in FP64 (oracle; test infrastructure).

Notation follows the paper (Sections 2-3): W weighted adjacency, d degrees,
D = diag(d), L = D - W, L_n = D^{-1/2} L D^{-1/2}, G group indicator,
F = first h-1 columns of F_0 = G - 1 z^T with z = G^T 1 / n (Lemma 2.1).

Two variants:
  * normalized (the paper's Alg. 3): min tr(H^T L H) s.t. H^T D H = I,
    F^T H = 0 (eq. normal-prob-fair), solved through X = D^{1/2} H,
    C = D^{-1/2} F.
  * unnormalized: the same derivation with D replaced by I in the
    constraint: min tr(H^T L H) s.t. H^T H = I, F^T H = 0, so C = F and
    H = X.  The paper states only the normalized algorithm; every proposition
    it proves carries over with L in place of L_n.

Tier A (dense, small n): explicit orthonormal nullspace basis Z of F^T from a
full QR (Alg. 2 step 2), then the dense (generalized) symmetric eigenproblem
on Z^T L Z (Alg. 2 steps 3-5 without the matrix square root, which only
changes variables).

Tier B (implicit, large n): the nullspace basis V of C^T kept as the h-1
Householder reflectors of a QR of C (FairSC variant 1, eq. lveig), and ARPACK
(scipy eigsh) on y -> V^T L_n V y.  No projector and no deflation: this is a
different route from the GPU method, which uses the deflated operator of
eq. asigma.

The deflated operator itself (eq. asigma and the matvec formula of Section
3.4 with P w = w - C z, z the least-squares solution of C z = w,
eq. mv-Pw) is also provided, for operator-level checks.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.linalg import lapack

__all__ = [
    "validate_graph",
    "degrees",
    "laplacian",
    "normalized_laplacian",
    "group_indicator",
    "fairness_matrix",
    "constraint_matrix",
    "shift_sigma",
    "fair_eigs_dense",
    "fair_eigs_implicit",
    "fair_eigs_deflated",
    "deflated_operator_dense",
    "apply_deflated_operator",
    "residual_norms",
]


def _as_csr(W) -> sp.csr_matrix:
    if sp.issparse(W):
        return sp.csr_matrix(W, dtype=np.float64)
    return sp.csr_matrix(np.asarray(W, dtype=np.float64))


def validate_graph(W, groups, h, k=None, normalized=False):
    """Check the paper's assumptions on the inputs (Section 2.1).

    W symmetric with w_ij >= 0 and w_ii = 0; every group non-empty (eq.
    groupdef); for the normalized variant no isolated vertex (D positive
    definite).  Raises ValueError naming the first violated assumption.
    """
    W = _as_csr(W)
    n = W.shape[0]
    if W.shape != (n, n):
        raise ValueError("W must be square")
    # finiteness first: a NaN makes every later comparison meaningless
    if not np.all(np.isfinite(W.data)):
        raise ValueError("non-finite weight")
    if W.nnz and W.data.min() < 0:
        raise ValueError("negative weight")
    if abs(W - W.T).max() != 0:
        raise ValueError("W is not symmetric")
    if np.any(W.diagonal() != 0):
        raise ValueError("non-zero diagonal")
    g = np.asarray(groups)
    if g.shape != (n,) or n == 0 or g.min() < 0 or g.max() >= h:
        raise ValueError("group labels out of range")
    if np.bincount(g, minlength=h).min() == 0:
        raise ValueError("empty group")
    if normalized and degrees(W).min() <= 0:
        raise ValueError("isolated vertex")
    if k is not None and not (1 <= k <= n - h + 1):
        raise ValueError("k out of range")


def degrees(W) -> np.ndarray:
    """d_i = sum_j w_ij (Section 2.1)."""
    return np.asarray(_as_csr(W).sum(axis=1)).ravel()


def laplacian(W) -> sp.csr_matrix:
    """L = D - W (eq. trace)."""
    W = _as_csr(W)
    return (sp.diags(degrees(W)) - W).tocsr()


def normalized_laplacian(W) -> sp.csr_matrix:
    """L_n = D^{-1/2} L D^{-1/2} (Alg. 1 step 2 / Alg. 3 step 2)."""
    W = _as_csr(W)
    s = 1.0 / np.sqrt(degrees(W))
    Ds = sp.diags(s)
    return (Ds @ laplacian(W) @ Ds).tocsr()


def group_indicator(groups, h) -> np.ndarray:
    """G in {0,1}^{n x h}, g_is = 1 iff v_i in V_s (eq. group-vec)."""
    g = np.asarray(groups)
    G = np.zeros((g.size, h))
    G[np.arange(g.size), g] = 1.0
    return G


def fairness_matrix(groups, h, drop=None) -> np.ndarray:
    """F of Lemma 2.1: F_0 = G - 1 z^T with z = G^T 1 / n, minus one column.

    By default the last column is dropped (the paper keeps the first h-1);
    `drop` selects another column, which by the lemma's footnote leaves the
    range, hence the projector, unchanged.
    """
    G = group_indicator(groups, h)
    n = G.shape[0]
    z = G.sum(axis=0) / n
    F0 = G - np.outer(np.ones(n), z)
    if drop is None:
        drop = h - 1
    keep = [s for s in range(h) if s != drop]
    return F0[:, keep]


def constraint_matrix(W, groups, h, normalized, drop=None) -> np.ndarray:
    """C = D^{-1/2} F (normalized, Section 3.2) or C = F (unnormalized)."""
    F = fairness_matrix(groups, h, drop)
    if normalized:
        return F / np.sqrt(degrees(W))[:, None]
    return F


def _operator_matrix(W, normalized):
    return normalized_laplacian(W) if normalized else laplacian(W)


def shift_sigma(W, normalized) -> float:
    """sigma = ||L_n||_1 (or ||L||_1), the shift the paper's experiments use
    (Appendix B.3, "Parameter sigma"): the largest absolute column sum."""
    A = _operator_matrix(W, normalized)
    return float(np.asarray(abs(A).sum(axis=0)).max())


def fair_eigs_dense(W, groups, h, k, normalized, drop=None):
    """Tier A: k smallest fair eigenpairs from an explicit nullspace basis.

    Alg. 2 steps 1-2 (L, and Z from a full QR of F, Section 3.1), then the
    trace minimisation of eq. normal-prob-fair-1 as the generalized symmetric
    eigenproblem (Z^T L Z) y = lambda (Z^T D Z) y for the normalized variant,
    or the standard one Z^T L Z y = lambda y for the unnormalized variant.
    Returns (lam[k] ascending, H n x k) with H = Z Y: F^T H = 0 and
    H^T D H = I (normalized) or H^T H = I (unnormalized).
    For h = 1 (no constraint) Z is the identity: plain SC (Alg. 1).
    """
    W = _as_csr(W)
    n = W.shape[0]
    L = laplacian(W).toarray()
    if h >= 2:
        F = fairness_matrix(groups, h, drop)
        Q, _ = np.linalg.qr(F, mode="complete")
        Z = Q[:, h - 1 :]
    else:
        Z = np.eye(n)
    M = Z.T @ L @ Z
    M = 0.5 * (M + M.T)
    if normalized:
        d = degrees(W)
        B = Z.T @ (d[:, None] * Z)
        B = 0.5 * (B + B.T)
        lam, Y = sla.eigh(M, B)
    else:
        lam, Y = np.linalg.eigh(M)
    H = Z @ Y[:, :k]
    return lam[:k].copy(), H


class _ImplicitNullspace:
    """V = orthonormal basis of null(C^T) held as Householder reflectors.

    From a QR of C (n x (h-1)): C = Q [R; 0], Q = H_1 ... H_{h-1}.  The last
    n-h+1 columns of Q span null(C^T), so V y = Q [0; y] and
    V^T x = (Q^T x)[h-1:] (FairSC variant 1; each apply is O(n h)).
    """

    def __init__(self, C):
        self.n, self.m = C.shape
        (self.qr, self.tau), _ = sla.qr(C, mode="raw")
        self.qr = np.asfortranarray(self.qr)

    def _apply(self, x, trans):
        x = np.asfortranarray(x.reshape(self.n, -1))
        lwork = max(1, x.shape[1]) * 64
        out, _, info = lapack.dormqr("L", trans, self.qr, self.tau, x, lwork)
        if info != 0:
            raise RuntimeError(f"dormqr info={info}")
        return out

    def V(self, y):
        y = np.asarray(y, dtype=np.float64).reshape(self.n - self.m, -1)
        full = np.zeros((self.n, y.shape[1]))
        full[self.m :] = y
        return self._apply(full, "N")

    def VT(self, x):
        return self._apply(np.asarray(x, dtype=np.float64), "T")[self.m :]


def fair_eigs_implicit(W, groups, h, k, normalized, tol=1e-12, seed=0, ncv=None, maxiter=None):
    """Tier B: k smallest fair eigenpairs without forming any n x n matrix.

    FairSC variant 1 (Section 3.2, eq. tropt_null and eq. lveig): the
    symmetric operator y -> V^T L_n V y (normalized, C = D^{-1/2} F) or
    y -> V^T L V y (unnormalized, C = F) on the (n-h+1)-dimensional nullspace,
    handed to ARPACK ("SA").  H = D^{-1/2} V y (normalized) or V y.
    Returns (lam[k] ascending, H n x k).
    """
    W = _as_csr(W)
    n = W.shape[0]
    A = _operator_matrix(W, normalized)
    if h >= 2:
        C = constraint_matrix(W, groups, h, normalized)
        ns = _ImplicitNullspace(C)
        dim = n - (h - 1)

        def mv(y):
            return ns.VT(A @ ns.V(y)).ravel()

        back = ns.V
    else:
        dim = n

        def mv(y):
            return A @ np.asarray(y).ravel()

        def back(y):
            return np.asarray(y).reshape(n, -1)

    op = spla.LinearOperator((dim, dim), matvec=mv, dtype=np.float64)
    rng = np.random.Generator(np.random.Philox(int(seed)))
    v0 = rng.standard_normal(dim)
    if ncv is None:
        ncv = min(dim, max(2 * k + 1, 4 * k, 40))
    lam, Y = spla.eigsh(op, k=k, which="SA", tol=tol, v0=v0, ncv=ncv, maxiter=maxiter)
    order = np.argsort(lam)
    lam = lam[order]
    X = back(Y[:, order])
    if normalized:
        X = X / np.sqrt(degrees(W))[:, None]
    return lam, X


def fair_eigs_deflated(W, groups, h, k, normalized, tol=1e-10, seed=0, ncv=None, sigma=None):
    """s-FairSC itself on the CPU (Alg. 3 step 3): ARPACK ("SA") on the
    deflated operator L^sigma applied by the matvec of Section 3.4
    (apply_deflated_operator); Proposition 3.3 makes its k smallest
    eigenpairs the fair ones.  H = D^{-1/2} X (normalized) or X.  This is
    the paper's own pipeline with a CPU eigensolver, timed beside the GPU
    library as the method-matched baseline.  Returns (lam[k], H n x k)."""
    W = _as_csr(W)
    n = W.shape[0]
    if sigma is None:
        sigma = shift_sigma(W, normalized)

    def mv(x):
        return apply_deflated_operator(W, groups, h, normalized, sigma, np.asarray(x).ravel())

    op = spla.LinearOperator((n, n), matvec=mv, dtype=np.float64)
    rng = np.random.Generator(np.random.Philox(int(seed)))
    if ncv is None:
        ncv = min(n, max(2 * k + 1, 4 * k, 40))
    lam, X = spla.eigsh(op, k=k, which="SA", tol=tol, v0=rng.standard_normal(n), ncv=ncv)
    order = np.argsort(lam)
    lam, X = lam[order], X[:, order]
    if normalized:
        X = X / np.sqrt(degrees(W))[:, None]
    return lam, X


def _projector_dense(C):
    """P = I - C (C^T C)^{-1} C^T (eq. pmat2 / eq. mv-Pw), via least squares."""
    n = C.shape[0]
    Z = np.linalg.lstsq(C, np.eye(n), rcond=None)[0]
    return np.eye(n) - C @ Z


def deflated_operator_dense(W, groups, h, normalized, sigma=None, drop=None):
    """L^sigma = P (L_n - sigma I) P + sigma I as a dense matrix (eq. asigma).

    sigma defaults to ||L_n||_1 (or ||L||_1 for the unnormalized variant).
    """
    A = _operator_matrix(W, normalized).toarray()
    n = A.shape[0]
    if sigma is None:
        sigma = shift_sigma(W, normalized)
    C = constraint_matrix(W, groups, h, normalized, drop)
    P = _projector_dense(C)
    return P @ (A - sigma * np.eye(n)) @ P + sigma * np.eye(n)


def apply_deflated_operator(W, groups, h, normalized, sigma, X):
    """Y = L^sigma X by the paper's matvec formula (Section 3.4 (i)-(ii)).

    L^sigma w = P(L_n (P w)) - sigma P w + sigma w, with P w = w - C z and z
    the least-squares solution of min ||C z - w||_2 (eq. mv-Pw), solved
    directly because h is small.  X is n x b (or a vector); FP64 throughout.
    """
    W = _as_csr(W)
    A = _operator_matrix(W, normalized)
    C = constraint_matrix(W, groups, h, normalized)
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    X2 = X.reshape(X.shape[0], -1)

    def P(w):
        z = np.linalg.lstsq(C, w, rcond=None)[0]
        return w - C @ z

    Pw = P(X2)
    Y = P(A @ Pw) - sigma * Pw + sigma * X2
    return Y.ravel() if vec else Y


def residual_norms(W, groups, h, normalized, lam, H):
    """Residuals of the fair eigenproblem for a computed (lam, H).

    With X = D^{1/2} H (normalized) or X = H, returns ||P L_n X_i - lam_i X_i||
    per column, the residual of the restricted operator V^T L_n V written in
    the original coordinates (exact eigenpairs give zero).
    """
    W = _as_csr(W)
    A = _operator_matrix(W, normalized)
    H = np.asarray(H, dtype=np.float64)
    X = H * np.sqrt(degrees(W))[:, None] if normalized else H
    C = constraint_matrix(W, groups, h, normalized)
    AX = A @ X
    z = np.linalg.lstsq(C, AX, rcond=None)[0]
    R = AX - C @ z - X * np.asarray(lam)[None, :]
    return np.linalg.norm(R, axis=0)
