"""A general constraint matrix F (sfairsc_graph_set_constraint) (GPU).

Inputs: the random-Laplacian workload (random sparse symmetric W, random
placeholder F; Section 5) and 0/1 group memberships, disjoint or
overlapping (Section 6).  The operator is compared element by element with
the oracle's least-squares projection (same tolerance reasoning as the
group operator: 1e-12 sigma max|X| in FP64, 2 (deg_max + 2) 2^-24 sigma
max|X| in mixed precision), eigenpairs with the oracle's dense route
(n = 700, several row tiles and a ragged tail) and, at the paper's
Experiment 4 size (n = 10,000, h = 5), with its implicit route and by
residuals.  A group matrix given as a general F must reproduce the group
path, and a rank-deficient F must give the rank of its range.
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_common import eig_parity, lib, log, to_np
from sfairsc_inputs import overlapping_memberships, random_laplacian, random_sparse_graph

pytestmark = pytest.mark.gpu


def _graph(sf, g, normalized, F=None, center=False, rank_tol=0.0):
    G = sf.Graph.from_msbm(g, normalized)
    r = None
    if F is not None:
        r = G.set_constraint(torch.from_numpy(np.ascontiguousarray(F)), center=center, rank_tol=rank_tol)
    return G, r


def _mixed_tol(g):
    return 2.0 * (int(np.diff(g.rowptr).max()) + 2) * 2.0**-24


@pytest.mark.parametrize("normalized", [False, True])
@pytest.mark.parametrize("m", [1, 4, 11])
@pytest.mark.parametrize("b", [1, 5, 8, 32])
def test_operator_matches_oracle(normalized, m, b):
    sf = lib()
    g, F = random_laplacian(700, 0.03, m, seed=31 + m)
    log(f"general operator n={g.n} nnz={g.nnz} m={m} b={b} normalized={normalized}")
    W = g.to_scipy()
    G, r = _graph(sf, g, normalized, F)
    assert r == m
    assert G.stats()["constraint_rank"] == m
    sigma = G.sigma
    X = np.random.default_rng(b + 7 * m).standard_normal((g.n, b))
    ref = oracle.apply_deflated_operator_general(W, F, normalized, sigma, X)
    scale = sigma * np.abs(X).max()
    Y = to_np(G.apply_operator(torch.from_numpy(X), "fp64"))
    assert np.abs(Y - ref).max() <= 1e-12 * scale
    Ym = to_np(G.apply_operator(torch.from_numpy(X), "mixed"))
    assert np.abs(Ym - ref).max() <= _mixed_tol(g) * scale


@pytest.mark.parametrize("normalized", [False, True])
def test_rank_deficient_F_gives_the_operator_of_its_range(normalized):
    sf = lib()
    g, F = random_laplacian(600, 0.04, 3, seed=40)
    rng = np.random.default_rng(2)
    Fd = np.concatenate([F, F @ rng.standard_normal((3, 2)), np.zeros((g.n, 1))], axis=1)
    G, r = _graph(sf, g, normalized, Fd)
    assert r == 3
    G0, r0 = _graph(sf, g, normalized, F)
    X = rng.standard_normal((g.n, 8))
    Y = to_np(G.apply_operator(torch.from_numpy(X)))
    Y0 = to_np(G0.apply_operator(torch.from_numpy(X)))
    ref = oracle.apply_deflated_operator_general(g.to_scipy(), Fd, normalized, G.sigma, X)
    scale = G.sigma * np.abs(X).max()
    assert np.abs(Y - Y0).max() <= 1e-12 * scale
    assert np.abs(Y - ref).max() <= 1e-12 * scale


@pytest.mark.parametrize("normalized", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_eigenpairs_match_the_dense_oracle(normalized, precision):
    sf = lib()
    g, F = random_laplacian(700, 0.03, 4, seed=33)
    W = g.to_scipy()
    k = 6
    lam, H, r = oracle.fair_eigs_dense_general(W, F, k + 1, normalized)
    assert r == 4
    G, rg = _graph(sf, g, normalized, F)
    tol = 1e-10 if precision == "fp64" else 1e-6
    res = G.eigs(k, tol=tol, precision=precision)
    err = eig_parity(res.eigenvalues, lam[:k], 0)
    log(f"general eigs normalized={normalized} {precision}: eigenvalue rel err {err:.2e}")
    assert err <= (1e-9 if precision == "fp64" else 1e-5)
    Hg = to_np(res.H)
    d = oracle.degrees(W)
    # F^T H = 0 and the D- (or plain) orthonormality hold to rounding
    assert np.abs(F.T @ Hg).max() <= 1e-10 * np.abs(F).max() * np.sqrt(g.n)
    B = Hg.T @ (d[:, None] * Hg) if normalized else Hg.T @ Hg
    assert np.abs(B - np.eye(k)).max() <= 1e-10
    gap = (lam[k] - lam[k - 1]) / lam[k]
    if gap > 1e-3:
        ang = oracle.max_principal_angle(Hg, H[:, :k], d if normalized else None)
        log(f"  subspace angle {ang:.2e} (relative gap {gap:.2e})")
        assert ang <= (1e-6 if precision == "fp64" else 1e-2)


@pytest.mark.parametrize("normalized", [False, True])
def test_group_matrix_reproduces_the_group_path(normalized):
    sf = lib()
    g = random_sparse_graph(900, 14, seed=35, h=3)
    k = 5
    Gg = sf.Graph.from_msbm(g, normalized)
    ref = Gg.eigs(k, tol=1e-11)
    # Lemma 2.1's F, and the one-hot memberships centred with every column kept
    Fl = oracle.fairness_matrix(g.groups, 3)
    G1, r1 = _graph(sf, g, normalized, Fl)
    onehot = np.eye(3)[g.groups]
    G2, r2 = _graph(sf, g, normalized, onehot, center=True)
    assert r1 == 2 and r2 == 2
    for G in (G1, G2):
        res = G.eigs(k, tol=1e-11)
        assert eig_parity(res.eigenvalues, ref.eigenvalues, 0) <= 1e-10
    lam, _ = oracle.fair_eigs_dense(g.to_scipy(), g.groups, 3, k, normalized)
    assert eig_parity(ref.eigenvalues, lam, 0) <= 1e-9


def test_overlapping_memberships():
    sf = lib()
    n, h = 800, 4
    g = random_sparse_graph(n, 16, seed=36, h=2)
    W = g.to_scipy()
    k = 5
    # union of two disjoint groups: an exact dependency, rank h - 1
    Gu = overlapping_memberships(n, h, 0.0, seed=5, union_of=(0, 1))
    Gv = overlapping_memberships(n, h, 0.25, seed=6)
    for memb, want in ((Gu, h - 1), (Gv, h)):
        F0 = oracle.membership_fairness_matrix(memb)
        lam, H, r = oracle.fair_eigs_dense_general(W, F0, k, True)
        assert r == want
        G, rg = _graph(sf, g, True, memb, center=True)
        assert rg == want
        res = G.eigs(k, tol=1e-10)
        err = eig_parity(res.eigenvalues, lam, 0)
        log(f"overlapping memberships rank {rg}: eigenvalue rel err {err:.2e}")
        assert err <= 1e-9
        assert np.abs(F0.T @ to_np(res.H)).max() <= 1e-10 * np.sqrt(n)


@pytest.mark.parametrize("normalized", [False, True])
def test_experiment4_size(normalized):
    # n = 10,000, h = 5 (m = 4 placeholder columns), k = 10
    sf = lib()
    g, F = random_laplacian(10000, 0.01, 4, seed=41)
    W = g.to_scipy()
    k = 10
    log(f"random Laplacian n={g.n} nnz={g.nnz} normalized={normalized}")
    lam, H, r = oracle.fair_eigs_implicit_general(W, F, k, normalized, tol=1e-12)
    G, rg = _graph(sf, g, normalized, F)
    assert rg == r == 4
    res = G.eigs(k, tol=1e-9, precision="mixed")
    log(f"  info {res.info}")
    err = eig_parity(res.eigenvalues, lam, 0)
    log(f"  eigenvalue rel err vs implicit oracle {err:.2e}")
    assert err <= 1e-8
    Hg = to_np(res.H)
    d = oracle.degrees(W)
    Lm = oracle.laplacian(W)
    # residual of the fair problem: the part of L h - lambda D h (or - lambda h)
    # outside range(F) vanishes at a fair eigenpair
    R = Lm @ Hg - (d[:, None] * Hg if normalized else Hg) * res.eigenvalues[None, :]
    Ur, _ = oracle.range_basis(F)
    R = R - Ur @ (Ur.T @ R)
    rel = np.linalg.norm(R, axis=0).max() / (G.sigma * (np.sqrt(d.max()) if normalized else 1.0))
    log(f"  projected residual / sigma {rel:.2e}")
    assert rel <= 1e-7
    assert np.abs(F.T @ Hg).max() <= 1e-10 * np.sqrt(g.n)


def test_batched_hands_general_handles_to_the_single_solver():
    sf = lib()
    gs = [random_laplacian(500 + 50 * i, 0.04, 3, seed=50 + i) for i in range(3)]
    Gs = [_graph(sf, g, True, F)[0] for g, F in gs]
    out = sf.eigs_batched(Gs, 4, tol=1e-9, precision="fp64")
    for (g, F), res in zip(gs, out):
        lam, _, _ = oracle.fair_eigs_dense_general(g.to_scipy(), F, 4, True)
        assert eig_parity(res.eigenvalues, lam, 0) <= 1e-8


def test_gradient_with_a_general_constraint():
    sf = lib()
    g, F = random_laplacian(400, 0.05, 3, seed=60)
    W = g.to_scipy()
    k = 4
    for normalized in (False, True):
        lam, H, _ = oracle.fair_eigs_dense_general(W, F, k + 1, normalized)
        assert (lam[k] - lam[k - 1]) / lam[k] > 1e-3
        G, _ = _graph(sf, g, normalized, F)
        res = G.eigs(k, tol=1e-12)
        grad = to_np(G.eigsum_backward(res.H, res.eigenvalues if normalized else None))
        if normalized:
            ref = oracle.eigsum_edge_gradient_normalized(g.rowptr, g.col, H[:, :k], lam[:k])
        else:
            ref = oracle.eigsum_edge_gradient(g.rowptr, g.col, H[:, :k])
        assert np.abs(grad - ref).max() <= 1e-8 * np.abs(ref).max()


def test_bad_constraints_are_rejected_and_the_group_constraint_returns():
    sf = lib()
    g = random_sparse_graph(300, 10, seed=61, h=2)
    G = sf.Graph.from_msbm(g, False)
    ref = G.eigs(3, tol=1e-10)
    F = np.random.default_rng(0).random((g.n, 40))
    for bad in (dict(F=F), dict(F=np.zeros((g.n, 2))), dict(F=F[:, :2], rank_tol=1e-9),
                dict(F=F[:, :2] * np.nan)):
        with pytest.raises(sf.SfairscError) as e:
            G.set_constraint(torch.from_numpy(np.ascontiguousarray(bad["F"])), rank_tol=bad.get("rank_tol", 0.0))
        assert e.value.code == sf.E_ARG
    assert G.stats()["constraint_rank"] == 1
    res = G.eigs(3, tol=1e-10)
    assert np.allclose(res.eigenvalues, ref.eigenvalues, rtol=1e-10)
    assert G.set_constraint(torch.from_numpy(F[:, :5].copy())) == 5
    assert G.stats()["constraint_rank"] == 5


def test_widest_constraint_and_padded_leading_dimension():
    # m = 32 columns (the widest basis), F stored with ldf > n
    sf = lib()
    import ctypes

    g, F = random_laplacian(900, 0.03, 32, seed=62)
    W = g.to_scipy()
    G = sf.Graph.from_msbm(g, True)
    ldf = g.n + 7
    Fp = np.zeros((32, ldf))
    Fp[:, : g.n] = F.T
    Fp[:, g.n:] = np.nan  # padding is never read
    Fd = torch.from_numpy(Fp).cuda()
    rank = ctypes.c_int32(0)
    code = sf._lib.lib().sfairsc_graph_set_constraint(G._h, ctypes.c_void_p(Fd.data_ptr()), ldf, 32, 0, 0.0,
                                                      ctypes.byref(rank), None)
    assert code == 0 and rank.value == 32
    X = np.random.default_rng(3).standard_normal((g.n, 8))
    ref = oracle.apply_deflated_operator_general(W, F, True, G.sigma, X)
    Y = to_np(G.apply_operator(torch.from_numpy(X)))
    assert np.abs(Y - ref).max() <= 1e-12 * G.sigma * np.abs(X).max()


def test_switching_between_constraint_forms():
    sf = lib()
    import scipy.sparse as sp

    g = random_sparse_graph(700, 14, seed=63, h=3)
    W = g.to_scipy()
    k = 4
    G = sf.Graph.from_msbm(g, True)
    ref = G.eigs(k, tol=1e-10).eigenvalues
    F = np.random.default_rng(4).random((g.n, 5))
    assert G.set_constraint(torch.from_numpy(F)) == 5
    lamF, _, _ = oracle.fair_eigs_dense_general(W, F, k, True)
    assert eig_parity(G.eigs(k, tol=1e-10).eigenvalues, lamF, 0) <= 1e-9
    M = overlapping_memberships(g.n, 6, 0.2, seed=5)
    G.set_memberships(sp.csr_matrix(M), inner_tol=1e-13)
    assert G.stats()["constraint_rank"] == 6
    lamM, _, _ = oracle.fair_eigs_dense_general(W, oracle.membership_fairness_matrix(M), k, True)
    assert eig_parity(G.eigs(k, tol=1e-10).eigenvalues, lamM, 0) <= 1e-9
    # back to the group matrix of Lemma 2.1 through the dense form
    assert G.set_constraint(torch.from_numpy(oracle.fairness_matrix(g.groups, 3))) == 2
    assert eig_parity(G.eigs(k, tol=1e-10).eigenvalues, ref, 0) <= 1e-9
