"""Pins of the general-F oracle (CPU): the group special case of Lemma 2.1,
the complete graph in closed form, invariance of the result under any change
of F that keeps its range, exact rank deficiency from overlapping groups,
agreement of the dense and implicit routes, and Propositions 3.1-3.2 for the
deflated operator."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from sfairsc_inputs import overlapping_memberships, random_laplacian, random_sparse_graph


def _angle(A, B):
    return oracle.max_principal_angle(A, B)


@pytest.mark.parametrize("normalized", [False, True])
def test_group_matrix_reduces_to_the_group_oracle(normalized):
    g = random_sparse_graph(80, 10, seed=21, h=3)
    W = g.to_scipy()
    k = 4
    lam0, H0 = oracle.fair_eigs_dense(W, g.groups, 3, k, normalized)
    F = oracle.fairness_matrix(g.groups, 3)
    lam, H, r = oracle.fair_eigs_dense_general(W, F, k, normalized)
    assert r == 2
    assert np.allclose(lam, lam0, rtol=1e-10, atol=1e-12)
    assert _angle(H, H0) < 1e-8
    # every column of the membership form: rank h - 1, same range
    G = np.eye(3)[g.groups]
    F0 = oracle.membership_fairness_matrix(G)
    assert np.allclose(F0.sum(axis=1), 0.0, atol=1e-14)
    lam1, H1, r1 = oracle.fair_eigs_dense_general(W, F0, k, normalized)
    assert r1 == 2
    assert np.allclose(lam1, lam0, rtol=1e-10, atol=1e-12)
    assert _angle(H1, H0) < 1e-8


def test_complete_graph_closed_form():
    # K_n: L = n I - 1 1^T.  On S = null(F^T) the form is n I - (Z^T 1)(Z^T 1)^T,
    # so lambda_1 = n - ||P_S 1||^2 = ||P_F 1||^2 = n - min_y ||1 - F y||^2 and
    # lambda_2 = ... = n.  The normalized pencil divides by d = n - 1.
    n = 30
    W = sp.csr_matrix(np.ones((n, n)) - np.eye(n))
    rng = np.random.default_rng(3)
    for F in (rng.random((n, 4)), np.concatenate([rng.random((n, 3)), np.zeros((n, 1))], axis=1)):
        F = np.concatenate([F, F[:, :2] @ np.array([[1.0], [-2.0]])], axis=1)  # a dependent column
        res = np.linalg.lstsq(F, np.ones(n), rcond=None)
        pf = n - float(np.sum((np.ones(n) - F @ res[0]) ** 2))
        lam, H, r = oracle.fair_eigs_dense_general(W, F, 3, False)
        assert r == np.linalg.matrix_rank(F)
        assert lam[0] == pytest.approx(pf, rel=1e-10)
        assert np.allclose(lam[1:], n, rtol=1e-12)
        lamn, _, _ = oracle.fair_eigs_dense_general(W, F, 3, True)
        assert np.allclose(lamn, lam / (n - 1), rtol=1e-10)


@pytest.mark.parametrize("normalized", [False, True])
def test_only_the_range_of_F_matters(normalized):
    g, F = random_laplacian(120, 0.08, 4, seed=5)
    W = g.to_scipy()
    k = 5
    lam, H, r = oracle.fair_eigs_dense_general(W, F, k, normalized)
    assert r == 4
    assert np.abs(F.T @ H).max() < 1e-10 * np.abs(H).max() * np.abs(F).max() * 120
    d = oracle.degrees(W)
    Bm = H.T @ (d[:, None] * H) if normalized else H.T @ H
    assert np.allclose(Bm, np.eye(k), atol=1e-10)
    rng = np.random.default_rng(8)
    M = rng.standard_normal((4, 4)) + 4 * np.eye(4)
    F2 = np.concatenate([F @ M, F @ rng.standard_normal((4, 2))], axis=1)
    lam2, H2, r2 = oracle.fair_eigs_dense_general(W, F2, k, normalized)
    assert r2 == 4
    assert np.allclose(lam2, lam, rtol=1e-10, atol=1e-12)
    assert _angle(H2, H) < 1e-7
    # Theorem 2.1: the fair minimum is at most tr(X^T L X) for any feasible X
    if not normalized:
        L = oracle.laplacian(W).toarray()
        Z = np.linalg.svd(F, full_matrices=True)[0][:, 4:]
        for _ in range(5):
            X, _ = np.linalg.qr(Z @ rng.standard_normal((Z.shape[1], k)))
            assert lam.sum() <= np.trace(X.T @ L @ X) + 1e-9


def test_union_group_is_an_exact_rank_deficiency():
    n, h = 90, 4
    g = random_sparse_graph(n, 12, seed=23, h=2)
    W = g.to_scipy()
    G = overlapping_memberships(n, h, 0.0, seed=2, union_of=(0, 1))
    assert G.shape == (n, h + 1) and G.sum(axis=1).max() == 2
    base = np.argmax(G[:, :h], axis=1).astype(np.int32)
    F0 = oracle.membership_fairness_matrix(G)
    for normalized in (False, True):
        lam, H, r = oracle.fair_eigs_dense_general(W, F0, 4, normalized)
        assert r == h - 1
        lam0, H0 = oracle.fair_eigs_dense(W, base, h, 4, normalized)
        assert np.allclose(lam, lam0, rtol=1e-10, atol=1e-12)
        assert _angle(H, H0) < 1e-7
    # overlapping memberships without the union: generically full rank h
    Go = overlapping_memberships(n, h, 0.3, seed=3)
    assert (Go.sum(axis=1) > 1).any()
    _, _, ro = oracle.fair_eigs_dense_general(W, oracle.membership_fairness_matrix(Go), 3, False)
    assert ro == h


@pytest.mark.parametrize("normalized", [False, True])
def test_implicit_route_agrees_with_the_dense_route(normalized):
    g, F = random_laplacian(300, 0.05, 4, seed=6)
    W = g.to_scipy()
    k = 6
    lam, H, r = oracle.fair_eigs_dense_general(W, F, k + 1, normalized)
    assert lam[k] - lam[k - 1] > 1e-4
    lam2, H2, r2 = oracle.fair_eigs_implicit_general(W, F, k, normalized, tol=1e-13)
    assert r2 == r == 4
    assert np.allclose(lam2, lam[:k], rtol=1e-9, atol=1e-12)
    assert _angle(H2, H[:, :k]) < 1e-6


@pytest.mark.parametrize("normalized", [False, True])
def test_operator_propositions(normalized):
    g, F = random_laplacian(150, 0.06, 3, seed=7)
    F = np.concatenate([F, F[:, :1] + F[:, 1:2]], axis=1)  # rank 3 of 4 columns
    W = g.to_scipy()
    sigma = oracle.shift_sigma(W, normalized)
    C = oracle.general_constraint_matrix(W, F, normalized)
    # Proposition 3.1: range(C) is an eigenspace of L^sigma with eigenvalue sigma
    Y = oracle.apply_deflated_operator_general(W, F, normalized, sigma, C)
    assert np.allclose(Y, sigma * C, atol=1e-10 * sigma * np.abs(C).max())
    # Proposition 3.2: a fair eigenpair (X = D^{1/2} H) is an eigenpair of L^sigma
    lam, H, r = oracle.fair_eigs_dense_general(W, F, 3, normalized)
    assert r == 3
    X = H * np.sqrt(oracle.degrees(W))[:, None] if normalized else H
    Y = oracle.apply_deflated_operator_general(W, F, normalized, sigma, X)
    assert np.allclose(Y, X * lam[None, :], atol=1e-9 * sigma * np.abs(X).max())
    # group F: the same numbers as the group-label operator of Section 3.4
    gg = random_sparse_graph(60, 8, seed=24, h=3)
    Wg = gg.to_scipy()
    s2 = oracle.shift_sigma(Wg, normalized)
    Xr = np.random.default_rng(1).standard_normal((60, 3))
    a = oracle.apply_deflated_operator(Wg, gg.groups, 3, normalized, s2, Xr)
    b = oracle.apply_deflated_operator_general(Wg, oracle.fairness_matrix(gg.groups, 3), normalized, s2, Xr)
    assert np.allclose(a, b, atol=1e-11 * s2 * np.abs(Xr).max())


@pytest.mark.parametrize("normalized", [False, True])
def test_gradient_formulas_hold_for_a_general_F(normalized):
    # F does not depend on W, so the envelope argument is unchanged
    g, F = random_laplacian(70, 0.15, 3, seed=9)
    n, k = 70, 4
    W = g.to_scipy()
    lam, H, _ = oracle.fair_eigs_dense_general(W, F, k + 1, normalized)
    assert (lam[k] - lam[k - 1]) / lam[k] > 1e-3
    if normalized:
        grad = oracle.eigsum_edge_gradient_normalized(g.rowptr, g.col, H[:, :k], lam[:k])
    else:
        grad = oracle.eigsum_edge_gradient(g.rowptr, g.col, H[:, :k])
    rows = g.row_index()
    rng = np.random.default_rng(4)
    step = 1e-6
    for e in rng.choice(np.flatnonzero(rows < g.col), 8, replace=False):
        i, j = int(rows[e]), int(g.col[e])
        vals = []
        for sgn in (1.0, -1.0):
            Wp = W.copy().tolil()
            Wp[i, j] += sgn * step
            Wp[j, i] += sgn * step
            vals.append(oracle.fair_eigs_dense_general(Wp.tocsr(), F, k, normalized)[0].sum())
        fd = (vals[0] - vals[1]) / (2 * step)
        mate = np.flatnonzero((rows == j) & (g.col == i))[0]
        assert grad[e] + grad[mate] == pytest.approx(fd, rel=1e-5, abs=1e-8)
