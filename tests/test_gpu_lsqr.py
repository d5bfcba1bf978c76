"""Membership constraints projected by LSQR (sfairsc_graph_set_memberships)
(GPU).

The inexact projection of Section 3.4 (ii) is checked against the exact
projection (the oracle's least-squares operator on the same C): the LSQR
stopping rule bounds the projection error by about inner_tol * cond(C) *
||r||, so with inner_tol = 1e-13 and cond(C) below 1e3 (computed here) the
operator must agree with the oracle to 1e-9 sigma max|X| in FP64.
Eigenpairs are compared with the oracle's dense and implicit routes for
memberships with m = 40 and m = 500 columns (more than the group path's
32 groups or the dense basis's 32 columns), overlapping groups included.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
from gpu_common import eig_parity, lib, log, to_np
from sfairsc_inputs import overlapping_memberships, random_sparse_graph

pytestmark = pytest.mark.gpu


def _cond(C):
    s = np.linalg.svd(C, compute_uv=False)
    s = s[s > 1e-10 * s[0]]
    return s[0] / s[-1]


def _mixed_tol(g):
    return 2.0 * (int(np.diff(g.rowptr).max()) + 2) * 2.0**-24


@pytest.mark.parametrize("normalized", [False, True])
@pytest.mark.parametrize("b", [1, 3, 8, 32])
def test_operator_matches_the_exact_projection(normalized, b):
    sf = lib()
    g = random_sparse_graph(1200, 12, seed=71, h=2)
    M = overlapping_memberships(g.n, 40, 0.3, seed=72)
    W = g.to_scipy()
    F0 = oracle.membership_fairness_matrix(M)
    C = oracle.general_constraint_matrix(W, F0, normalized)
    kappa = _cond(C)
    log(f"lsqr operator n={g.n} m=40 b={b} normalized={normalized} cond(C)={kappa:.1f}")
    assert kappa < 1e3
    G = sf.Graph.from_msbm(g, normalized)
    G.set_memberships(M, center=True, inner_tol=1e-13)
    assert G.stats()["constraint_rank"] == 40
    sigma = G.sigma
    X = np.random.default_rng(b).standard_normal((g.n, b))
    ref = oracle.apply_deflated_operator_general(W, F0, normalized, sigma, X)
    scale = sigma * np.abs(X).max()
    Y = to_np(G.apply_operator(torch.from_numpy(X), "fp64"))
    err = np.abs(Y - ref).max() / scale
    log(f"  fp64 max error / (sigma max|X|) {err:.2e}")
    assert err <= 1e-9
    Ym = to_np(G.apply_operator(torch.from_numpy(X), "mixed"))
    assert np.abs(Ym - ref).max() <= _mixed_tol(g) * scale + 1e-9 * scale
    st = G.lsqr_stats()
    log(f"  lsqr {st}")
    assert st["solves"] == 4 and st["unconverged"] == 0
    assert st["max_steps"] < 200


@pytest.mark.parametrize("normalized", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_eigenpairs_with_overlapping_memberships(normalized, precision):
    sf = lib()
    g = random_sparse_graph(1200, 12, seed=73, h=2)
    M = overlapping_memberships(g.n, 40, 0.3, seed=74)
    W = g.to_scipy()
    F0 = oracle.membership_fairness_matrix(M)
    k = 5
    lam, H, r = oracle.fair_eigs_dense_general(W, F0, k, normalized)
    assert r == 40
    G = sf.Graph.from_msbm(g, normalized)
    G.set_memberships(M, inner_tol=1e-13)
    tol = 1e-9 if precision == "fp64" else 1e-6
    res = G.eigs(k, tol=tol, precision=precision)
    err = eig_parity(res.eigenvalues, lam, 0)
    log(f"lsqr eigs normalized={normalized} {precision}: rel err {err:.2e} info {res.info}")
    assert err <= (1e-8 if precision == "fp64" else 1e-5)
    Hg = to_np(res.H)
    # the fair output is projected once more: F^T H = 0 to the inner tolerance
    assert np.abs(F0.T @ Hg).max() <= 1e-9 * np.sqrt(g.n)
    st = G.lsqr_stats()
    log(f"  lsqr {st}")
    assert st["unconverged"] == 0


@pytest.mark.parametrize("normalized", [False, True])
def test_one_hot_memberships_reproduce_the_group_path(normalized):
    sf = lib()
    g = random_sparse_graph(900, 14, seed=75, h=3)
    k = 5
    ref = sf.Graph.from_msbm(g, normalized).eigs(k, tol=1e-10)
    G = sf.Graph.from_msbm(g, normalized)
    G.set_memberships(sp.csr_matrix(np.eye(3)[g.groups]), center=True, inner_tol=1e-14)
    res = G.eigs(k, tol=1e-10)
    assert eig_parity(res.eigenvalues, ref.eigenvalues, 0) <= 1e-9


def test_many_groups():
    # m = 500 groups (each vertex in 1 or 2), n = 10,000
    sf = lib()
    g = random_sparse_graph(10000, 20, seed=76, h=2)
    M = overlapping_memberships(g.n, 500, 0.2, seed=77)
    W = g.to_scipy()
    F0 = oracle.membership_fairness_matrix(M)
    k = 8
    lam, H, r = oracle.fair_eigs_implicit_general(W, F0, k, True, tol=1e-12)
    G = sf.Graph.from_msbm(g, True)
    G.set_memberships(sp.csr_matrix(M), inner_tol=1e-12)
    res = G.eigs(k, tol=1e-8, precision="mixed")
    err = eig_parity(res.eigenvalues, lam, 0)
    st = G.lsqr_stats()
    log(f"many groups: rank {r}, rel err {err:.2e}, info {res.info}, lsqr {st}")
    assert err <= 1e-7
    assert st["unconverged"] == 0
    Hg = to_np(res.H)
    assert np.abs(F0.T @ Hg).max() <= 1e-8 * np.sqrt(g.n)


def test_batched_hands_membership_handles_to_the_single_solver():
    sf = lib()
    gs = [random_sparse_graph(600 + 40 * i, 12, seed=80 + i, h=2) for i in range(2)]
    Ms = [overlapping_memberships(g.n, 35, 0.2, seed=90 + i) for i, g in enumerate(gs)]
    Gs = []
    for g, M in zip(gs, Ms):
        G = sf.Graph.from_msbm(g, False)
        G.set_memberships(M, inner_tol=1e-13)
        Gs.append(G)
    out = sf.eigs_batched(Gs, 4, tol=1e-9, precision="fp64")
    for g, M, res in zip(gs, Ms, out):
        lam, _, _ = oracle.fair_eigs_dense_general(g.to_scipy(), oracle.membership_fairness_matrix(M), 4, False)
        assert eig_parity(res.eigenvalues, lam, 0) <= 1e-8


def test_bad_memberships_are_rejected():
    sf = lib()
    g = random_sparse_graph(300, 10, seed=81, h=2)
    G = sf.Graph.from_msbm(g, False)
    with pytest.raises(sf.SfairscError):
        G.lsqr_stats()
    M = overlapping_memberships(g.n, 4, 0.1, seed=82)
    for kw in (dict(inner_tol=1e-20), dict(inner_tol=2.0), dict(max_inner=-1)):
        with pytest.raises(sf.SfairscError) as e:
            G.set_memberships(M, **kw)
        assert e.value.code == sf.E_ARG
    # a column index out of range and a repeated membership
    Mc = sp.csr_matrix(M)
    bad = Mc.copy()
    bad.indices = bad.indices.copy()
    bad.indices[0] = 7
    rp = torch.from_numpy(bad.indptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(bad.indices.astype(np.int32)).cuda()
    lib_ = sf._lib.lib()
    import ctypes

    code = lib_.sfairsc_graph_set_memberships(G._h, 4, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(ci.data_ptr()),
                                              1, 0.0, 0, None)
    assert code == sf.E_ARG
    rows = np.diff(Mc.indptr)
    i = int(np.flatnonzero(rows >= 2)[0])
    dup = Mc.indices.copy()
    dup[Mc.indptr[i] + 1] = dup[Mc.indptr[i]]
    ci2 = torch.from_numpy(dup.astype(np.int32)).cuda()
    rp2 = torch.from_numpy(Mc.indptr.astype(np.int32)).cuda()
    code = lib_.sfairsc_graph_set_memberships(G._h, 4, ctypes.c_void_p(rp2.data_ptr()),
                                              ctypes.c_void_p(ci2.data_ptr()), 1, 0.0, 0, None)
    assert code == sf.E_ARG
    # the group constraint applies again
    assert G.stats()["constraint_rank"] == 1


def test_uncentred_memberships_and_an_unused_group():
    # F = G without centring; group 7 has no member (a zero column of C)
    sf = lib()
    g = random_sparse_graph(800, 12, seed=83, h=2)
    W = g.to_scipy()
    M = overlapping_memberships(g.n, 7, 0.25, seed=84)
    M8 = np.concatenate([M, np.zeros((g.n, 1))], axis=1)
    for normalized in (False, True):
        G = sf.Graph.from_msbm(g, normalized)
        G.set_memberships(sp.csr_matrix(M8), center=False, inner_tol=1e-13)
        X = np.random.default_rng(5).standard_normal((g.n, 4))
        ref = oracle.apply_deflated_operator_general(W, M8, normalized, G.sigma, X)
        Y = to_np(G.apply_operator(torch.from_numpy(X)))
        assert np.abs(Y - ref).max() <= 1e-9 * G.sigma * np.abs(X).max()
        lam, _, r = oracle.fair_eigs_dense_general(W, M8, 4, normalized)
        assert r == 7
        res = G.eigs(4, tol=1e-9)
        assert eig_parity(res.eigenvalues, lam, 0) <= 1e-8


def test_step_cap_is_reported():
    sf = lib()
    g = random_sparse_graph(600, 12, seed=85, h=2)
    M = overlapping_memberships(g.n, 30, 0.3, seed=86)
    G = sf.Graph.from_msbm(g, False)
    G.set_memberships(sp.csr_matrix(M), inner_tol=1e-14, max_inner=2)
    X = torch.from_numpy(np.random.default_rng(6).standard_normal((g.n, 3)))
    G.apply_operator(X)
    st = G.lsqr_stats()
    assert st["solves"] == 2 and st["max_steps"] == 2 and st["unconverged"] > 0
