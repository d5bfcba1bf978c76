"""Pins of the FP64 oracle against what the paper and mathematics fix (CPU only).

Each test checks the oracle against something other than itself: a value the
paper prints, a closed-form spectrum, an invariant stated by a proposition, a
special case that reduces to a textbook routine, or the minimum property of
the trace problem.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from conftest import read_golden
from sfairsc_inputs import msbm_from_blocks, random_sparse_graph, workload
from sfairsc_inputs.msbm import fair_block_sizes


def _cycle(n):
    i = np.arange(n)
    j = (i + 1) % n
    W = sp.coo_matrix((np.ones(n), (i, j)), shape=(n, n))
    return (W + W.T).tocsr()


def _complete(n):
    W = np.ones((n, n)) - np.eye(n)
    return sp.csr_matrix(W)


# --- Lemma 2.1 ---------------------------------------------------------------


@pytest.mark.parametrize("h", [2, 3, 5, 6])
def test_lemma21_rank(h):
    rng = np.random.default_rng(h)
    g = rng.integers(0, h, 40)
    g[:h] = np.arange(h)
    G = oracle.group_indicator(g, h)
    z = G.sum(0) / 40
    F0 = G - np.outer(np.ones(40), z)
    assert np.linalg.matrix_rank(F0) == h - 1
    assert np.linalg.matrix_rank(oracle.fairness_matrix(g, h)) == h - 1


def test_example_b2_fairness_matrix_and_fair_H():
    gold = read_golden("example_b2_msbm.txt")
    g1 = np.array(list(map(float, gold["g1"])))
    groups = (1 - g1).astype(int)  # group 0 = V_1
    F = oracle.fairness_matrix(groups, 2)
    # z = (5/10, 5/10), F = g^(1) - 1/2 (Lemma 2.1 with h = 2)
    assert np.array_equal(F[:, 0], g1 - 0.5)
    H = np.stack([np.array(list(map(float, gold[f"H_col{c}"]))) for c in (1, 2, 3)], 1)
    assert np.array_equal(F.T @ H, np.zeros((1, 3)))  # the planted clustering is fair
    # an unfair clustering violates F^T H = 0 (Lemma 2.1 (ii))
    bad = np.zeros((10, 2))
    bad[:3, 0] = 1
    bad[3:, 1] = 1
    assert np.abs(F.T @ bad).max() > 0


def test_column_choice_does_not_change_projector():
    # footnote to Lemma 2.1: any h-1 columns of F_0 give the same range
    g = random_sparse_graph(60, 8, seed=2, h=4)
    W = g.to_scipy()
    A0 = oracle.deflated_operator_dense(W, g.groups, 4, True, drop=0)
    A3 = oracle.deflated_operator_dense(W, g.groups, 4, True, drop=3)
    assert np.abs(A0 - A3).max() < 1e-12


# --- closed-form spectra -------------------------------------------------------


@pytest.mark.parametrize("n", [8, 12, 30])
def test_cycle_with_alternating_groups(n):
    # L(C_n) has eigenvalues 2 - 2 cos(2 pi j / n); with groups i mod 2 the
    # constraint vector F = +-1/2 alternating is the j = n/2 eigenvector
    # (eigenvalue 4), so the fair spectrum drops exactly one copy of 4.
    W = _cycle(n)
    groups = np.arange(n) % 2
    full = np.sort(2 - 2 * np.cos(2 * np.pi * np.arange(n) / n))
    expect = np.delete(full, np.argmin(np.abs(full - 4.0)))
    lam, H = oracle.fair_eigs_dense(W, groups, 2, n - 1, False)
    assert np.allclose(lam, expect, atol=1e-12)
    lamB, _ = oracle.fair_eigs_implicit(W, groups, 2, 4, False)
    assert np.allclose(lamB, expect[:4], atol=1e-10)


@pytest.mark.parametrize("normalized", [False, True])
def test_complete_graph(normalized):
    # L(K_n) = n I - 1 1^T: eigenvalue 0 once (vector 1, which is fair) and n
    # otherwise; L_n = I - (1 1^T - I)/(n-1): 0 and n/(n-1).
    n, h = 12, 3
    groups = np.arange(n) % h
    lam, _ = oracle.fair_eigs_dense(_complete(n), groups, h, n - h + 1, normalized)
    top = n / (n - 1) if normalized else float(n)
    assert abs(lam[0]) < 1e-12
    assert np.allclose(lam[1:], top, atol=1e-12)


def test_disjoint_fair_cliques_give_k_zero_eigenvalues():
    # k disjoint cliques, each exactly fair: the fair eigenvalue 0 has
    # multiplicity k and its eigenspace is spanned by the clique indicators
    # (the eigenspace-mixing case of Section 3.3).
    k, per = 3, 4
    n = k * per
    W = np.zeros((n, n))
    for c in range(k):
        W[c * per : (c + 1) * per, c * per : (c + 1) * per] = 1
    np.fill_diagonal(W, 0)
    groups = np.arange(n) % 2
    for normalized in (False, True):
        lam, H = oracle.fair_eigs_dense(sp.csr_matrix(W), groups, 2, k + 1, normalized)
        assert np.all(np.abs(lam[:k]) < 1e-12)
        assert lam[k] > 0.5
        ind = np.kron(np.eye(k), np.ones((per, 1)))
        d = W.sum(1) if normalized else None
        assert oracle.max_principal_angle(H[:, :k], ind, d) < 1e-10


@pytest.mark.parametrize("normalized", [False, True])
def test_trivial_pair(normalized):
    # F^T 1 = 0, so 1 is feasible and L 1 = 0: lambda_1 = 0 with H ~ 1
    g = workload("msbm-500-h4-grad")
    W = g.to_scipy()
    lam, H = oracle.fair_eigs_dense(W, g.groups, g.h, 3, normalized)
    assert abs(lam[0]) < 1e-12
    v = H[:, 0] / np.linalg.norm(H[:, 0])
    assert abs(abs(v @ np.ones(g.n)) / np.sqrt(g.n) - 1) < 1e-12


# --- special cases reducing to textbook routines ----------------------------------


def test_h1_is_plain_spectral_clustering():
    # without groups the problem is Alg. 1: eigenvectors of L_n, H = D^{-1/2} X
    g = random_sparse_graph(80, 10, seed=4, h=2)
    W = g.to_scipy()
    d = oracle.degrees(W)
    Ln = np.eye(80) - W.toarray() / np.sqrt(np.outer(d, d))
    mu, X = np.linalg.eigh(Ln)
    lam, H = oracle.fair_eigs_dense(W, np.zeros(80, int), 1, 5, True)
    assert np.allclose(lam, mu[:5], atol=1e-12)
    assert oracle.max_principal_angle(H[:, 1:5], X[:, 1:5] / np.sqrt(d)[:, None], d) < 1e-8


# --- Propositions 3.1 - 3.3 -------------------------------------------------------


@pytest.mark.parametrize("normalized", [False, True])
def test_deflated_spectrum(normalized):
    # spec(L^sigma) = spec(L^v) U {sigma}^(h-1) (Props. 3.1 and 3.2), and the
    # sigma-eigenvectors span range(C)
    g = random_sparse_graph(70, 9, seed=5, h=4)
    W = g.to_scipy()
    n, h = 70, 4
    sigma = oracle.shift_sigma(W, normalized)
    A = oracle.deflated_operator_dense(W, g.groups, h, normalized, sigma)
    assert np.abs(A - A.T).max() < 1e-12
    mu, U = np.linalg.eigh(A)
    lam, _ = oracle.fair_eigs_dense(W, g.groups, h, n - h + 1, normalized)
    expect = np.sort(np.concatenate([lam, np.full(h - 1, sigma)]))
    assert np.allclose(mu, expect, atol=1e-10 * sigma)
    C = oracle.constraint_matrix(W, g.groups, h, normalized)
    near = np.abs(mu - sigma) < 1e-8 * sigma
    # the sigma-eigenspace contains range(C) (it may be larger if some
    # lambda_i happens to equal sigma; not the case here)
    assert near.sum() == h - 1
    assert oracle.max_principal_angle(U[:, near], C) < 1e-8


@pytest.mark.parametrize("normalized", [False, True])
def test_prop33_two_formulations_agree(normalized):
    # the k smallest eigenvectors of L^sigma give the fair solution exactly
    g = workload("msbm-500-h4-grad")
    W = g.to_scipy()
    k = 6
    lam, H = oracle.fair_eigs_dense(W, g.groups, g.h, k, normalized)
    A = oracle.deflated_operator_dense(W, g.groups, g.h, normalized)
    mu, X = np.linalg.eigh(A)
    assert np.allclose(mu[:k], lam, rtol=1e-10, atol=1e-11)
    d = oracle.degrees(W)
    Hs = X[:, :k] / np.sqrt(d)[:, None] if normalized else X[:, :k]
    gap = lam[k - 1]
    assert oracle.max_principal_angle(Hs, H, d if normalized else None) < 1e-8


@pytest.mark.parametrize("normalized", [False, True])
def test_tier_a_outputs_satisfy_constraints(normalized):
    g = workload("msbm-500-h4-grad")
    W = g.to_scipy()
    lam, H = oracle.fair_eigs_dense(W, g.groups, g.h, 8, normalized)
    F = oracle.fairness_matrix(g.groups, g.h)
    d = oracle.degrees(W)
    assert np.abs(F.T @ H).max() < 1e-12 * np.abs(F).max() * np.abs(H).max() * g.n
    M = H.T @ (d[:, None] * H) if normalized else H.T @ H
    assert np.abs(M - np.eye(8)).max() < 1e-11
    # Theorem 2.1: tr(H^T L H) = sum of the eigenvalues
    L = oracle.laplacian(W)
    assert np.trace(H.T @ (L @ H)) == pytest.approx(lam.sum(), rel=1e-11)
    assert oracle.residual_norms(W, g.groups, g.h, normalized, lam, H).max() < 1e-10


@pytest.mark.parametrize("normalized", [False, True])
def test_trace_minimum_property(normalized):
    # Theorem 2.1: no feasible H (F^T H = 0, H^T D H = I) has a smaller trace
    g = random_sparse_graph(90, 10, seed=6, h=3)
    W = g.to_scipy()
    k = 4
    lam, _ = oracle.fair_eigs_dense(W, g.groups, 3, k, normalized)
    L = oracle.laplacian(W).toarray()
    F = oracle.fairness_matrix(g.groups, 3)
    d = oracle.degrees(W) if normalized else np.ones(90)
    rng = np.random.default_rng(0)
    P = np.eye(90) - F @ np.linalg.solve(F.T @ F, F.T)
    for _ in range(20):
        Y = P @ rng.standard_normal((90, k))
        R = np.linalg.cholesky(Y.T @ (d[:, None] * Y))
        Y = Y @ np.linalg.inv(R).T
        assert np.trace(Y.T @ L @ Y) >= lam.sum() - 1e-10


def test_sigma_closed_forms():
    g = workload("msbm-500-h4-grad")
    W = g.to_scipy()
    d = oracle.degrees(W)
    assert oracle.shift_sigma(W, False) == pytest.approx(2 * d.max(), rel=1e-14)
    what = W.multiply(1 / np.sqrt(np.outer(d, d)) if False else 1.0)
    s = 1 / np.sqrt(d)
    rows = np.asarray((sp.diags(s) @ W @ sp.diags(s)).sum(1)).ravel()
    assert oracle.shift_sigma(W, True) == pytest.approx(1 + rows.max(), rel=1e-14)


# --- the operator ----------------------------------------------------------------


@pytest.mark.parametrize("normalized", [False, True])
def test_operator_on_range_and_eigenvectors(normalized):
    g = random_sparse_graph(120, 9, seed=8, h=3)
    W = g.to_scipy()
    sigma = oracle.shift_sigma(W, normalized)
    C = oracle.constraint_matrix(W, g.groups, 3, normalized)
    # range(C) is the sigma-eigenspace: L^sigma C = sigma C
    Y = oracle.apply_deflated_operator(W, g.groups, 3, normalized, sigma, C)
    assert np.abs(Y - sigma * C).max() < 1e-12 * sigma
    lam, H = oracle.fair_eigs_dense(W, g.groups, 3, 5, normalized)
    d = oracle.degrees(W)
    X = H * np.sqrt(d)[:, None] if normalized else H
    Y = oracle.apply_deflated_operator(W, g.groups, 3, normalized, sigma, X)
    assert np.abs(Y - X * lam).max() < 1e-10 * sigma
    # matches the dense form of eq. asigma on random vectors
    Z = np.random.default_rng(1).standard_normal((120, 3))
    A = oracle.deflated_operator_dense(W, g.groups, 3, normalized, sigma)
    assert np.abs(A @ Z - oracle.apply_deflated_operator(W, g.groups, 3, normalized, sigma, Z)).max() < 1e-11 * sigma


# --- Tier B against Tier A ------------------------------------------------------


@pytest.mark.parametrize("normalized", [False, True])
def test_tier_b_matches_tier_a(normalized):
    g = workload("msbm-2k-h2")
    W = g.to_scipy()
    k = 6
    lamA, HA = oracle.fair_eigs_dense(W, g.groups, g.h, k, normalized)
    lamB, HB = oracle.fair_eigs_implicit(W, g.groups, g.h, k, normalized)
    scale = oracle.shift_sigma(W, normalized)
    assert np.allclose(lamA, lamB, rtol=1e-10, atol=1e-11 * scale)
    d = oracle.degrees(W) if normalized else None
    assert oracle.max_principal_angle(HA[:, :5], HB[:, :5], d) < 1e-7


@pytest.mark.parametrize("normalized", [False, True])
def test_cpu_sfairsc_pipeline_matches_tier_a(normalized):
    # Proposition 3.3: the k smallest eigenpairs of the deflated operator are
    # the fair ones (the CPU pipeline timed as the method-matched baseline)
    g = workload("msbm-2k-h2")
    W = g.to_scipy()
    k = 6
    lamA, HA = oracle.fair_eigs_dense(W, g.groups, g.h, k, normalized)
    lamS, HS = oracle.fair_eigs_deflated(W, g.groups, g.h, k, normalized)
    scale = oracle.shift_sigma(W, normalized)
    assert np.allclose(lamA, lamS, rtol=1e-10, atol=1e-11 * scale)
    d = oracle.degrees(W) if normalized else None
    assert oracle.max_principal_angle(HA[:, :5], HS[:, :5], d) < 1e-7
    # the deflated eigenvalue sigma stays out of the k smallest
    assert lamS.max() < 0.9 * scale


# --- planted recovery (Section 4, Experiment 1) ---------------------------------


def test_planted_recovery_where_sc_fails():
    # With the paper's ordering (same-group links across clusters more likely
    # than cross-group links inside a cluster), SC finds the groups instead of
    # the clusters, while fair SC recovers the planted fair clusters.
    n, k, h = 1000, 5, 5
    s = (np.log(n) / n) ** (2 / 3)
    u = fair_block_sizes([n // k] * k, [1] * h)
    g = msbm_from_blocks(u, (10 * s, 4 * s, 7 * s, 1 * s), seed=21)
    W = g.to_scipy()
    _, Hf = oracle.fair_eigs_dense(W, g.groups, h, k, True)
    lab_f, _ = oracle.kmeans(Hf, k, 10, 0)
    _, Hs = oracle.fair_eigs_dense(W, np.zeros(n, int), 1, k, True)
    lab_s, _ = oracle.kmeans(Hs, k, 10, 0)
    assert oracle.error_rate(lab_f, g.clusters) < 0.01
    assert oracle.error_rate(lab_s, g.clusters) > 0.3


def test_planted_recovery_small_workload():
    g = workload("msbm-2k-h2")
    lam, H = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, 5, False)
    lab, _ = oracle.kmeans(H, 5, 10, 0)
    assert oracle.error_rate(lab, g.clusters) == 0.0
    assert oracle.average_balance(lab, g.groups, 2, 5) == 1.0
