"""Pins of the oracle's LSQR (CPU): the exact least-squares solution and
projection, finite termination on a well-conditioned problem, agreement with
an independent implementation (scipy's lsqr), the minimum-norm solution and
the exact projection for a rank-deficient C, the stopping rule, and the
trivial right-hand sides."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle


def _problem(n=200, m=6, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, m)), rng.standard_normal(n)


def test_exact_least_squares_solution_and_projection():
    C, w = _problem()
    x, it, test = oracle.lsqr(lambda v: C @ v, lambda u: C.T @ u, w, atol=1e-14)
    ref = np.linalg.lstsq(C, w, rcond=None)[0]
    assert np.allclose(x, ref, rtol=1e-10, atol=1e-12)
    # finite termination: m steps in exact arithmetic, a couple more here
    assert it <= C.shape[1] + 3
    P = np.eye(C.shape[0]) - C @ np.linalg.pinv(C)
    Pw, _, _ = oracle.project_lsqr(C, w[:, None], atol=1e-14)
    assert np.allclose(Pw[:, 0], P @ w, atol=1e-12 * np.linalg.norm(w))
    # the residual is orthogonal to range(C)
    assert np.abs(C.T @ Pw).max() <= 1e-11 * np.linalg.norm(w) * np.abs(C).max()


def test_agrees_with_scipy_lsqr():
    rng = np.random.default_rng(1)
    C = rng.random((300, 12)) @ np.diag(np.logspace(0, 2, 12))  # kappa about 1e3
    w = rng.standard_normal(300)
    x, it, _ = oracle.lsqr(lambda v: C @ v, lambda u: C.T @ u, w, atol=1e-13, maxiter=500)
    xs = spla.lsqr(C, w, atol=1e-13, btol=1e-13, iter_lim=500)[0]
    assert np.allclose(x, xs, rtol=1e-8, atol=1e-10 * np.abs(xs).max())


def test_rank_deficient_gives_minimum_norm_and_the_projection():
    rng = np.random.default_rng(2)
    B = rng.standard_normal((150, 4))
    C = np.concatenate([B, B[:, :2] @ rng.standard_normal((2, 3)), np.zeros((150, 1))], axis=1)
    w = rng.standard_normal(150)
    x, it, test = oracle.lsqr(lambda v: C @ v, lambda u: C.T @ u, w, atol=1e-14)
    assert np.allclose(x, np.linalg.pinv(C) @ w, rtol=1e-8, atol=1e-10)
    U = np.linalg.svd(B, full_matrices=False)[0]
    Pw, _, _ = oracle.project_lsqr(C, w, atol=1e-14)
    assert np.allclose(Pw, w - U @ (U.T @ w), atol=1e-12 * np.linalg.norm(w))


@pytest.mark.parametrize("atol", [1e-4, 1e-8])
def test_stopping_rule_holds_on_exit(atol):
    rng = np.random.default_rng(3)
    C = rng.random((400, 30)) @ np.diag(np.logspace(0, 3, 30))
    w = rng.standard_normal(400)
    x, it, test = oracle.lsqr(lambda v: C @ v, lambda u: C.T @ u, w, atol=atol, maxiter=1000)
    r = w - C @ x
    ratio = np.linalg.norm(C.T @ r) / (np.linalg.norm(C) * np.linalg.norm(r))
    assert test <= atol
    # the estimate tracks the true quantity (Frobenius norm bound: the
    # estimate's ||C||_est never exceeds ||C||_F)
    assert ratio <= 10 * atol


def test_trivial_right_hand_sides():
    C, _ = _problem(50, 3, seed=4)
    x, it, _ = oracle.lsqr(lambda v: C @ v, lambda u: C.T @ u, np.zeros(50))
    assert it == 0 and not x.any()
    # w orthogonal to range(C): z = 0 and P w = w exactly
    Q = np.linalg.qr(np.concatenate([C, np.random.default_rng(5).standard_normal((50, 1))], axis=1))[0]
    w = Q[:, 3]
    x, it, _ = oracle.lsqr(lambda v: C @ v, lambda u: C.T @ u, w)
    assert np.abs(x).max() <= 1e-15 * 50
    Pw, _, _ = oracle.project_lsqr(C, w)
    assert np.allclose(Pw, w, atol=1e-14)


def test_membership_constraint_matrix():
    from sfairsc_inputs import overlapping_memberships, random_sparse_graph

    g = random_sparse_graph(120, 10, seed=7, h=2)
    W = g.to_scipy()
    G = overlapping_memberships(120, 5, 0.2, seed=8)
    for normalized in (False, True):
        C = oracle.membership_constraint_matrix(W, G, normalized)
        F0 = G - G.mean(axis=0)[None, :]
        d = oracle.degrees(W)
        assert np.allclose(C, F0 / np.sqrt(d)[:, None] if normalized else F0, atol=1e-15)
