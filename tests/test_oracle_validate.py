"""Pins of the oracle's input validation and of its residual measure (CPU only).

`validate_graph` restates the assumptions of Section 2.1 (w_ij = w_ji >= 0,
w_ii = 0) and eq. groupdef (h non-empty groups), plus the two conditions
the method adds: D positive definite for the normalized variant (Alg. 3
step 2 needs D^{-1/2}) and 1 <= k <= n - h + 1 (the constrained space
null(F^T) has dimension n - h + 1, Lemma 2.1).  Every branch is fed one
input that violates exactly that assumption, and the message names it.

`residual_norms` is the main acceptance measure of the full-size GPU tests,
so it is pinned on both sides: zero on exact fair eigenpairs, and the exact
non-zero value on pairs perturbed in ways whose residual is known in
closed form.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from sfairsc_inputs import random_sparse_graph


def _base(n=40, h=3, seed=3):
    g = random_sparse_graph(n, 6, seed=seed, h=h)
    return g.to_scipy().tocsr(), g.groups.copy(), h


def _raises(match, W, groups, h, **kw):
    with pytest.raises(ValueError, match=match):
        oracle.validate_graph(W, groups, h, **kw)


# --- validate_graph ---------------------------------------------------------


def test_valid_inputs_pass():
    W, g, h = _base()
    oracle.validate_graph(W, g, h)
    oracle.validate_graph(W, g, h, k=1, normalized=True)
    oracle.validate_graph(W, g, h, k=W.shape[0] - h + 1)


def test_asymmetric_value():
    W, g, h = _base()
    W = W.tolil()
    i, j = W.nonzero()[0][0], W.nonzero()[1][0]
    W[i, j] = W[i, j] + 0.25
    _raises("not symmetric", W.tocsr(), g, h)


def test_asymmetric_pattern():
    W, g, h = _base()
    W = W.tolil()
    # an entry stored on one side only
    i, j = next((a, b) for a in range(40) for b in range(40) if a != b and W[a, b] == 0)
    W[i, j] = 1.0
    _raises("not symmetric", W.tocsr(), g, h)


@pytest.mark.parametrize("bad, msg", [(-1.0, "negative"), (np.nan, "non-finite"), (np.inf, "non-finite"),
                                      (-np.inf, "non-finite")])
def test_bad_weight_symmetric(bad, msg):
    W, g, h = _base()
    W = W.tolil()
    i, j = W.nonzero()[0][0], W.nonzero()[1][0]
    W[i, j] = bad
    W[j, i] = bad
    _raises(msg, W.tocsr(), g, h)


def test_nonzero_diagonal():
    W, g, h = _base()
    W = W.tolil()
    W[5, 5] = 1.0
    _raises("diagonal", W.tocsr(), g, h)


@pytest.mark.parametrize("label", [-1, 3, 7])
def test_group_label_out_of_range(label):
    W, g, h = _base()
    g[4] = label
    _raises("out of range", W, g, h)


def test_group_labels_wrong_length():
    W, g, h = _base()
    _raises("out of range", W, g[:-1], h)


def test_empty_group():
    W, g, h = _base()
    g[g == 1] = 0
    _raises("empty group", W, g, h)


def test_isolated_vertex_only_rejected_when_normalized():
    W, g, h = _base()
    W = W.tolil()
    for j in list(W.rows[0]):
        W[0, j] = 0.0
        W[j, 0] = 0.0
    W = W.tocsr()
    W.eliminate_zeros()
    oracle.validate_graph(W, g, h, normalized=False)
    _raises("isolated", W, g, h, normalized=True)


@pytest.mark.parametrize("k", [0, -2, 39, 100])
def test_k_out_of_range(k):
    # n = 40, h = 3: the constrained space has dimension 38
    W, g, h = _base()
    _raises("k out of range", W, g, h, k=k)


def test_not_square():
    W = sp.csr_matrix(np.ones((3, 4)))
    _raises("square", W, np.zeros(3, int), 1)


# --- residual_norms -----------------------------------------------------------


@pytest.mark.parametrize("normalized", [False, True])
def test_residual_zero_on_exact_pairs(normalized):
    W, g, h = _base(60, 3, 11)
    lam, H = oracle.fair_eigs_dense(W, g, h, 6, normalized)
    r = oracle.residual_norms(W, g, h, normalized, lam, H)
    assert r.max() < 1e-12 * oracle.shift_sigma(W, normalized)


@pytest.mark.parametrize("normalized", [False, True])
def test_residual_of_a_shifted_eigenvalue(normalized):
    # (lambda_i + delta, h_i): r = delta x_i with ||x_i|| = 1 in the plain
    # inner product (x = D^{1/2} h for the normalized form)
    W, g, h = _base(60, 3, 12)
    lam, H = oracle.fair_eigs_dense(W, g, h, 5, normalized)
    delta = np.array([1e-3, -2e-2, 0.5, 3.0, -7.0])
    r = oracle.residual_norms(W, g, h, normalized, lam + delta, H)
    assert np.allclose(r, np.abs(delta), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("normalized", [False, True])
def test_residual_of_a_mixed_eigenvector(normalized):
    # (lambda_i, h_i + eps h_j): the restricted operator maps x_j to
    # lambda_j x_j, so r = eps |lambda_j - lambda_i| ||x_j|| = eps |lambda_j - lambda_i|
    W, g, h = _base(60, 4, 13)
    lam, H = oracle.fair_eigs_dense(W, g, h, 6, normalized)
    eps = 1e-3
    Hp = H.copy()
    pairs = [(0, 3), (1, 5), (2, 0), (4, 1)]
    lam_p = np.array([lam[i] for i, _ in pairs])
    Hp = np.stack([H[:, i] + eps * H[:, j] for i, j in pairs], 1)
    r = oracle.residual_norms(W, g, h, normalized, lam_p, Hp)
    want = np.array([eps * abs(lam[j] - lam[i]) for i, j in pairs])
    assert np.allclose(r, want, rtol=1e-8, atol=1e-13)


def test_residual_of_a_range_component():
    # (lambda_i, x_i + c) with c in range(C): r = || P L c - lambda_i c ||.
    # For the complete graph L = n I - 1 1^T and 1^T c = 0 (F^T 1 = 0), so
    # L c = n c lies in range(C) and P L c = 0: r = lambda_i ||c||.  An
    # oracle that skipped the projection would give (n - lambda_i) ||c||.
    n, h = 12, 3
    W = sp.csr_matrix(np.ones((n, n)) - np.eye(n))
    g = np.arange(n) % h
    lam, H = oracle.fair_eigs_dense(W, g, h, 3, False)
    assert np.allclose(lam, [0.0, n, n], atol=1e-12)
    F = oracle.fairness_matrix(g, h)
    c = 1e-2 * F[:, 0]
    r = oracle.residual_norms(W, g, h, False, lam, H + c[:, None])
    assert np.allclose(r, np.abs(lam) * np.linalg.norm(c), rtol=1e-10, atol=1e-14)
