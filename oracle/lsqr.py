"""LSQR for the projection's least-squares problem (oracle; test
infrastructure).

Section 3.4 (ii) writes P w = w - C z with z the least-squares solution of
min ||C z - w||_2 (eq. mv-Pw) and, for large problems, suggests an
iterative solver such as LSQR (Paige and Saunders, ACM TOMS 8, 1982) inside
the eigensolver (an inner-outer iteration).  This module restates LSQR from
its published recurrences (Golub-Kahan bidiagonalisation started from w,
Givens rotations of the bidiagonal, the solution update along the search
direction), one right-hand side at a time, in plain FP64 numpy.

Stopping rule (the second of Paige and Saunders' tests): stop when the estimate
||C^T r|| = phi_bar alpha |c| falls to atol * ||C||_est * ||r||, with
||C||_est the Frobenius norm of the bidiagonal built so far, or after
maxiter steps, or on an exact breakdown (alpha or beta zero).
"""

from __future__ import annotations

import numpy as np

__all__ = ["lsqr", "project_lsqr", "membership_constraint_matrix"]


def lsqr(matvec, rmatvec, w, atol=1e-12, maxiter=200):
    """x approximately minimising ||A x - w||_2 from x_0 = 0.

    matvec(v) = A v, rmatvec(u) = A^T u.  Returns (x, iterations,
    estimate of ||A^T r|| / (||A||_est ||r||) at exit)."""
    w = np.asarray(w, dtype=np.float64)
    beta = np.linalg.norm(w)
    x = None
    if beta == 0.0:
        return np.zeros_like(rmatvec(w)), 0, 0.0
    u = w / beta
    v = rmatvec(u)
    alpha = np.linalg.norm(v)
    x = np.zeros_like(v)
    if alpha == 0.0:
        return x, 0, 0.0
    v = v / alpha
    d = v.copy()  # search direction
    phi_bar, rho_bar = beta, alpha
    anorm2 = alpha * alpha
    test = np.inf
    it = 0
    while it < maxiter:
        it += 1
        # bidiagonalisation step
        u = matvec(v) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0.0:
            u = u / beta
        v_next = rmatvec(u) - beta * v
        alpha = np.linalg.norm(v_next)
        if alpha > 0.0:
            v_next = v_next / alpha
        anorm2 += alpha * alpha + beta * beta
        # rotation eliminating beta
        rho = np.hypot(rho_bar, beta)
        c, s = rho_bar / rho, beta / rho
        theta = s * alpha
        rho_bar = -c * alpha
        phi = c * phi_bar
        phi_bar = s * phi_bar
        # update of the solution and the direction
        x = x + (phi / rho) * d
        d = v_next - (theta / rho) * d
        v = v_next
        rnorm = phi_bar
        arnorm = phi_bar * alpha * abs(c)
        test = arnorm / (np.sqrt(anorm2) * rnorm) if rnorm > 0 else 0.0
        if test <= atol or alpha == 0.0 or beta == 0.0:
            break
    return x, it, test


def project_lsqr(C, W, atol=1e-12, maxiter=200):
    """P~ W = W - C z per column, z from lsqr (C n x m dense).  Returns
    (P~W, Z, iterations per column)."""
    C = np.asarray(C, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    W2 = W.reshape(W.shape[0], -1)
    Z = np.zeros((C.shape[1], W2.shape[1]))
    its = []
    for j in range(W2.shape[1]):
        z, it, _ = lsqr(lambda v: C @ v, lambda u: C.T @ u, W2[:, j], atol, maxiter)
        Z[:, j] = z
        its.append(it)
    return (W2 - C @ Z).reshape(W.shape), Z, its


def membership_constraint_matrix(W, G, normalized):
    """C = D^{-1/2} (G - 1 z^T) (normalized) or G - 1 z^T, z = G^T 1 / n, for a
    0/1 membership matrix G (dense or scipy sparse, n x m, every column kept;
    overlapping memberships allowed)."""
    from .general_f import general_constraint_matrix, membership_fairness_matrix

    G = G.toarray() if hasattr(G, "toarray") else np.asarray(G, dtype=np.float64)
    return general_constraint_matrix(W, membership_fairness_matrix(G), normalized)
