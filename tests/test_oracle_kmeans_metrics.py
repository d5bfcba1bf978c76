"""Pins of the oracle's k-means, random stream, metrics and gradient (CPU only)."""

import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from conftest import read_golden
from oracle.kmeans import kmeans_pp_seeds, lloyd
from sfairsc_inputs import random_sparse_graph, workload


def test_splitmix64_published_vectors():
    gold = read_golden("splitmix64_vectors.txt")
    assert oracle.splitmix64_outputs(1234567, 5) == [int(x) for x in gold["seed_1234567"]]
    assert oracle.splitmix64_outputs(0, 3) == [int(x, 16) for x in gold["seed_0"]]


def test_uniform_stream_is_in_range_and_uniform():
    u = np.array([oracle.splitmix64_uniform(5, r, t) for r in range(4) for t in range(2000)])
    assert u.min() >= 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 0.01


def _blobs(rng, k, per, dim, spread=0.05):
    centers = rng.standard_normal((k, dim)) * 3
    X = np.concatenate([c + spread * rng.standard_normal((per, dim)) for c in centers])
    truth = np.repeat(np.arange(k), per)
    return X, truth


def _all_partitions_inertia(X, k):
    n = X.shape[0]
    best = np.inf
    for lab in itertools.product(range(k), repeat=n):
        lab = np.array(lab)
        if len(set(lab)) != k:
            continue
        tot = 0.0
        for j in range(k):
            P = X[lab == j]
            tot += ((P - P.mean(0)) ** 2).sum()
        best = min(best, tot)
    return best


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kmeans_finds_bruteforce_optimum(seed):
    rng = np.random.default_rng(seed)
    X, _ = _blobs(rng, 3, 3, 2, spread=0.3)
    lab, inertia = oracle.kmeans(X, 3, 10, seed)
    assert inertia == pytest.approx(_all_partitions_inertia(X, 3), rel=1e-12)


def test_kmeans_recovers_blobs_and_is_rotation_invariant():
    rng = np.random.default_rng(3)
    X, truth = _blobs(rng, 5, 40, 5)
    lab, _ = oracle.kmeans(X, 5, 10, 0)
    assert oracle.same_partition(lab, truth)
    Q, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    lab2, _ = oracle.kmeans(X @ Q, 5, 10, 0)
    assert np.array_equal(lab, lab2)


def test_kmeanspp_first_seed_and_distinct():
    X = np.random.default_rng(0).standard_normal((97, 3))
    idx = kmeans_pp_seeds(X, 6, seed=11, restart=2)
    assert idx[0] == int(oracle.splitmix64_uniform(11, 2, 0) * 97)
    assert len(set(idx)) == 6


def test_kmeans_degenerate_points():
    # all points identical: D^2 total is 0, clusters empty -> still valid labels
    X = np.ones((7, 2))
    lab, inertia = oracle.kmeans(X, 3, 2, 0)
    assert inertia == 0.0 and lab.shape == (7,) and lab.min() >= 0 and lab.max() < 3
    # an empty cluster is refilled with the farthest point
    X = np.array([[0.0], [0.1], [10.0], [10.1], [50.0]])
    lab, inertia, it = lloyd(X, np.array([[0.0], [10.0], [1000.0]]))
    assert len(set(lab.tolist())) == 3


def test_error_rate_matches_bruteforce_and_paper_scale():
    rng = np.random.default_rng(0)
    for k in (2, 3, 4, 5):
        truth = rng.integers(0, k, 40)
        pred = rng.integers(0, k, 40)
        assert oracle.error_rate(pred, truth, k) == pytest.approx(oracle.error_rate_bruteforce(pred, truth, k))
    # four vertices, one misclustered: the literal eq. err gives 2/4
    truth = np.array([0, 0, 1, 1])
    pred = np.array([1, 1, 0, 1])
    assert oracle.error_rate(pred, truth, 2) == 0.25
    assert oracle.error_rate_bruteforce(pred, truth, 2, paper_scale=True) == 0.5


def test_balance_bound_and_zero():
    groups = np.array([0] * 30 + [1] * 20)
    fair = np.concatenate([np.arange(30) % 2, np.arange(20) % 2])
    # a fair clustering attains the bound min |V_s| / |V_s'| (eq. bal-upper)
    assert np.allclose(oracle.balance(fair, groups, 2, 2), 20 / 30)
    unfair = np.array([0] * 30 + [1] * 20)
    assert np.all(oracle.balance(unfair, groups, 2, 2) == 0)
    rng = np.random.default_rng(1)
    for _ in range(20):
        lab = rng.integers(0, 3, 50)
        assert oracle.balance(lab, groups, 2, 3).min() <= 20 / 30 + 1e-15


def test_principal_angle_known_rotation():
    th = 0.3
    A = np.zeros((5, 2))
    A[0, 0] = A[1, 1] = 1
    B = A.copy()
    B[:, 1] = np.cos(th) * A[:, 1]
    B[2, 1] = np.sin(th)
    assert oracle.max_principal_angle(A, B) == pytest.approx(th, rel=1e-12)


# --- gradient of the eigenvalue sum -------------------------------------------


def _edge_list(g):
    rows = g.row_index()
    up = rows < g.col
    return rows[up], g.col[up], g.val[up].astype(np.float64)


def _eigsum(n, ei, ej, w, groups, h, k):
    W = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([ei, ej]), np.concatenate([ej, ei]))), shape=(n, n)).tocsr()
    lam, _ = oracle.fair_eigs_dense(W, groups, h, k, False)
    return lam.sum()


def test_gradient_matches_finite_differences():
    g = random_sparse_graph(60, 10, seed=9, h=3)
    k = 4
    W = g.to_scipy()
    lam, H = oracle.fair_eigs_dense(W, g.groups, 3, k + 1, False)
    assert lam[k] - lam[k - 1] > 1e-3
    grad = oracle.eigsum_edge_gradient(g.rowptr, g.col, H[:, :k])
    ei, ej, w = _edge_list(g)
    rows = g.row_index()
    step = 1e-6
    rng = np.random.default_rng(0)
    for e in rng.choice(ei.size, 12, replace=False):
        wp = w.copy()
        wp[e] += step
        wm = w.copy()
        wm[e] -= step
        fd = (_eigsum(60, ei, ej, wp, g.groups, 3, k) - _eigsum(60, ei, ej, wm, g.groups, 3, k)) / (2 * step)
        i, j = ei[e], ej[e]
        a = np.flatnonzero((rows == i) & (g.col == j))[0]
        b = np.flatnonzero((rows == j) & (g.col == i))[0]
        assert grad[a] + grad[b] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def _eigsum_csr(W, groups, h, k, normalized):
    lam, _ = oracle.fair_eigs_dense(W, groups, h, k, normalized)
    return lam.sum()


def test_normalized_gradient_matches_finite_differences():
    # edges (both stored copies perturbed together) and stored diagonal
    # entries (perturbed alone: they enter D but not L)
    g = random_sparse_graph(60, 10, seed=11, h=3)
    n, k = 60, 4
    W = g.to_scipy().tolil()
    for i in (3, 17, 40):
        W[i, i] = 0.7
    W = W.tocsr()
    W.sort_indices()
    rowptr, col = W.indptr.astype(np.int64), W.indices.astype(np.int64)
    lam, H = oracle.fair_eigs_dense(W, g.groups, 3, k + 1, True)
    assert lam[k] - lam[k - 1] > 1e-3
    d = oracle.degrees(W)
    assert np.allclose(H.T @ (d[:, None] * H), np.eye(k + 1), atol=1e-10)
    grad = oracle.eigsum_edge_gradient_normalized(rowptr, col, H[:, :k], lam[:k])
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    rng = np.random.default_rng(1)
    off = np.flatnonzero(rows < col)
    picks = [(int(rows[e]), int(col[e])) for e in rng.choice(off, 10, replace=False)] + [(3, 3), (17, 17), (40, 40)]
    step = 1e-6
    for i, j in picks:
        Wp, Wm = W.copy().tolil(), W.copy().tolil()
        Wp[i, j] += step
        Wm[i, j] -= step
        if i != j:
            Wp[j, i] += step
            Wm[j, i] -= step
        fd = (_eigsum_csr(Wp.tocsr(), g.groups, 3, k, True) - _eigsum_csr(Wm.tocsr(), g.groups, 3, k, True)) / (2 * step)
        a = np.flatnonzero((rows == i) & (col == j))[0]
        b = np.flatnonzero((rows == j) & (col == i))[0]
        an = grad[a] + (grad[b] if i != j else 0.0)
        assert an == pytest.approx(fd, rel=1e-5, abs=1e-8), (i, j)
    # the unnormalized formula misses the degree term: it must not pass here
    plain = oracle.eigsum_edge_gradient(rowptr, col, H[:, :k])
    assert np.abs(plain - grad).max() > 1e-3 * np.abs(grad).max()


def test_normalized_gradient_matches_autograd_of_dense_generalized_eigh():
    torch = pytest.importorskip("torch")
    g = random_sparse_graph(50, 8, seed=12, h=2)
    k = 3
    ei, ej, w = _edge_list(g)
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    n = 50
    Wd = torch.zeros((n, n), dtype=torch.float64)
    Wd = Wd.index_put((torch.tensor(ei), torch.tensor(ej)), wt, accumulate=True)
    Wd = Wd + Wd.T
    d = Wd.sum(1)
    L = torch.diag(d) - Wd
    F = torch.tensor(oracle.fairness_matrix(g.groups, 2))
    Q, _ = torch.linalg.qr(F, mode="complete")
    Z = Q[:, 1:]
    M = Z.T @ L @ Z
    B = Z.T @ (d[:, None] * Z)
    C = torch.linalg.cholesky(0.5 * (B + B.T))
    Ci = torch.linalg.inv(C)
    S = Ci @ (0.5 * (M + M.T)) @ Ci.T
    lam = torch.linalg.eigvalsh(0.5 * (S + S.T))
    lam[:k].sum().backward()
    lamo, H = oracle.fair_eigs_dense(g.to_scipy(), g.groups, 2, k, True)
    assert np.allclose(lamo, lam[:k].detach().numpy(), rtol=1e-10, atol=1e-12)
    grad = oracle.eigsum_edge_gradient_normalized(g.rowptr, g.col, H, lamo)
    rows = g.row_index()
    lookup = {(int(r), int(c)): t for t, (r, c) in enumerate(zip(rows, g.col))}
    per_edge = np.array([grad[lookup[(ei[e], ej[e])]] + grad[lookup[(ej[e], ei[e])]] for e in range(ei.size)])
    assert np.allclose(per_edge, wt.grad.numpy(), rtol=1e-8, atol=1e-10)


def test_gradient_matches_autograd_of_dense_eigh():
    torch = pytest.importorskip("torch")
    g = random_sparse_graph(50, 8, seed=10, h=2)
    k = 3
    ei, ej, w = _edge_list(g)
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    n = 50
    Wd = torch.zeros((n, n), dtype=torch.float64)
    Wd = Wd.index_put((torch.tensor(ei), torch.tensor(ej)), wt, accumulate=True)
    Wd = Wd + Wd.T
    L = torch.diag(Wd.sum(1)) - Wd
    F = torch.tensor(oracle.fairness_matrix(g.groups, 2))
    Q, _ = torch.linalg.qr(F, mode="complete")
    Z = Q[:, 1:]
    M = Z.T @ L @ Z
    lam = torch.linalg.eigvalsh(0.5 * (M + M.T))
    lam[:k].sum().backward()
    _, H = oracle.fair_eigs_dense(g.to_scipy(), g.groups, 2, k, False)
    grad = oracle.eigsum_edge_gradient(g.rowptr, g.col, H)
    rows = g.row_index()
    per_edge = np.zeros(ei.size)
    lookup = {(int(r), int(c)): t for t, (r, c) in enumerate(zip(rows, g.col))}
    for e in range(ei.size):
        per_edge[e] = grad[lookup[(ei[e], ej[e])]] + grad[lookup[(ej[e], ei[e])]]
    assert np.allclose(per_edge, wt.grad.numpy(), rtol=1e-8, atol=1e-10)
