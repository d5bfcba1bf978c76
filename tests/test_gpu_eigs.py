"""Parity of the fair eigensolver (sfairsc_eigs) against the FP64 oracle (GPU).

Bars (Proposition 3.3 makes the GPU's eigenpairs of L^sigma the fair
eigenpairs the oracle computes from an explicit nullspace):
  * eigenvalues: relative 1e-8 in FP64, 1e-5 for the mixed solve; the
    trivial eigenvalue 0 is compared against lambda_2;
  * subspace: largest principal angle (D-weighted for the normalized
    variant) <= 1e-6 (FP64) / 1e-4 (mixed), asserted only when the relative
    gap (lambda_{k+1} - lambda_k) / sigma exceeds 100 tol (Davis-Kahan);
  * constraints: F^T H = 0, H^T H = I (or H^T D H = I), and the oracle's own
    residual of every returned pair below the requested tolerance.
"""

import os

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
from conftest import read_golden
from gpu_common import eig_parity, lib, log, to_np
from sfairsc_inputs import msbm_from_blocks, random_sparse_graph, relabel, workload

pytestmark = pytest.mark.gpu


def check_solution(g, lam, H, k, normalized, tol, sigma, lam_ref=None, H_ref=None, rtol=1e-8, atol_angle=1e-6,
                   gap=None):
    W = g.to_scipy()
    d = oracle.degrees(W)
    F = oracle.fairness_matrix(g.groups, g.h) if g.h > 1 else np.zeros((g.n, 0))
    Hn = H
    assert np.all(np.diff(lam) >= -1e-12 * sigma), "eigenvalues not ascending"
    if F.shape[1]:
        assert np.abs(F.T @ Hn).max() <= 1e-10 * np.sqrt(g.n) * np.abs(Hn).max()
    M = Hn.T @ (d[:, None] * Hn) if normalized else Hn.T @ Hn
    assert np.abs(M - np.eye(k)).max() <= 1e-9
    # the library returns only pairs whose FP64 residual ||L^sigma x - theta x||
    # meets tol sigma; for x in null(C^T) that residual is exactly the
    # oracle's ||P L x - theta x||, so only rounding separates the two
    res = oracle.residual_norms(W, g.groups, g.h, normalized, lam, Hn)
    assert res.max() <= tol * sigma + 2e-12 * sigma, res.max() / sigma
    if lam_ref is not None:
        err = eig_parity(lam, lam_ref[:k], rtol)
        log(f"  eigenvalue rel err {err:.2e}")
        assert err <= rtol
    if H_ref is not None and gap is not None and gap > 100 * tol:
        ang = oracle.max_principal_angle(Hn, H_ref[:, :k], d if normalized else None)
        log(f"  subspace angle {ang:.2e}")
        assert ang <= atol_angle


@pytest.mark.parametrize("normalized", [False, True])
def test_msbm_2k_fp64(normalized):
    sf = lib()
    g = workload("msbm-2k-h2")
    k, tol = 5, 1e-10
    log(f"msbm-2k fp64 normalized={normalized}")
    lam_ref, H_ref = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, k + 1, normalized)
    G = sf.Graph.from_msbm(g, normalized)
    r = G.eigs(k, tol=tol, precision="fp64")
    log(f"  info {r.info}")
    sigma = G.sigma
    gap = (lam_ref[k] - lam_ref[k - 1]) / sigma
    check_solution(g, r.eigenvalues, to_np(r.H), k, normalized, tol, sigma, lam_ref, H_ref, 1e-8, 1e-6, gap)
    # planted recovery with the GPU k-means
    lab, _ = G.labels(r.H, 5, n_restarts=10, seed=0)
    assert oracle.error_rate(to_np(lab), g.clusters) == 0.0


@pytest.mark.parametrize("normalized", [False, True])
def test_msbm_2k_mixed(normalized):
    sf = lib()
    g = workload("msbm-2k-h2")
    k, tol = 5, 1e-8
    log(f"msbm-2k mixed normalized={normalized}")
    lam_ref, H_ref = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, k + 1, normalized)
    G = sf.Graph.from_msbm(g, normalized)
    r = G.eigs(k, tol=tol, precision="mixed")
    log(f"  info {r.info}")
    sigma = G.sigma
    gap = (lam_ref[k] - lam_ref[k - 1]) / sigma
    check_solution(g, r.eigenvalues, to_np(r.H), k, normalized, tol, sigma, lam_ref, H_ref, 1e-5, 1e-4, gap)
    assert r.info["spmm_launches"][1] > 0


def test_relabelled_graph():
    sf = lib()
    g = relabel(workload("msbm-2k-h2"), 17)
    k, tol = 5, 1e-10
    lam_ref, H_ref = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, k + 1, False)
    G = sf.Graph.from_msbm(g, False)
    r = G.eigs(k, tol=tol)
    gap = (lam_ref[k] - lam_ref[k - 1]) / G.sigma
    check_solution(g, r.eigenvalues, to_np(r.H), k, False, tol, G.sigma, lam_ref, H_ref, 1e-8, 1e-6, gap)


SMALL = [
    (97, 8, 1, 2, False, 3),
    (97, 8, 2, 2, True, 2),
    (250, 12, 3, 3, False, 4),
    (250, 12, 4, 3, True, 6),
    (613, 6, 5, 1, False, 5),
    (613, 6, 6, 2, True, 4),
    (1201, 20, 7, 4, False, 8),
]


@pytest.mark.parametrize("case", SMALL, ids=[f"n{c[0]}-h{c[3]}-{'norm' if c[4] else 'unnorm'}" for c in SMALL])
def test_small_random_graphs(case):
    sf = lib()
    n, deg, seed, h, normalized, k = case
    g = random_sparse_graph(n, deg, seed=seed, h=h, weights=("uniform", 0.5, 1.5))
    log(f"small graph {case}")
    lam_ref, H_ref = oracle.fair_eigs_dense(g.to_scipy(), g.groups, h, k + 1, normalized)
    G = sf.Graph.from_msbm(g, normalized)
    tol = 1e-10
    r = G.eigs(k, tol=tol)
    gap = (lam_ref[k] - lam_ref[k - 1]) / G.sigma
    check_solution(g, r.eigenvalues, to_np(r.H), k, normalized, tol, G.sigma, lam_ref, H_ref, 1e-8, 1e-6, gap)


# The solver's operator is the reassociated form T = L X - (L C) U_in (one
# L C term in the first orthogonalisation pass).  These cases drive each of its
# kernel variants: up to four constraint columns from quad broadcasts, more
# (h > 5) with the extended tail, block widths 4 and 16 (one column tile) and
# 32 (two tiles), FP64 and mixed, both Laplacians.
REASSOC = [
    (900, 10, 21, 7, True, 4, 8, "fp64"),
    (900, 10, 22, 6, False, 5, 16, "fp64"),
    (1400, 12, 23, 9, True, 3, 4, "mixed"),
    (1400, 12, 24, 5, False, 6, 32, "fp64"),
    (1100, 8, 25, 3, True, 4, 16, "mixed"),
    (1600, 10, 26, 5, True, 5, 4, "fp64"),
    # many groups: the last orthogonalisation pass forms the operator's input
    # group sums in two 16-group tiles (h > 16), up to the maximum of 32
    (2000, 12, 27, 24, True, 5, 8, "fp64"),
    (2000, 12, 28, 32, False, 4, 4, "fp64"),
    (2000, 12, 29, 32, True, 5, 8, "mixed"),
]


@pytest.mark.parametrize("case", REASSOC, ids=[f"h{c[3]}-b{c[6]}-{c[7]}-{'norm' if c[4] else 'unnorm'}" for c in REASSOC])
def test_reassociated_operator_paths(case):
    sf = lib()
    n, deg, seed, h, normalized, k, b, prec = case
    g = random_sparse_graph(n, deg, seed=seed, h=h, weights=("uniform", 0.5, 1.5))
    log(f"reassociated operator {case}")
    lam_ref, H_ref = oracle.fair_eigs_dense(g.to_scipy(), g.groups, h, k + 1, normalized)
    G = sf.Graph.from_msbm(g, normalized)
    tol = 1e-10 if prec == "fp64" else 1e-8
    r = G.eigs(k, tol=tol, precision=prec, block_width=b)
    gap = (lam_ref[k] - lam_ref[k - 1]) / G.sigma
    rtol, ang = (1e-8, 1e-6) if prec == "fp64" else (1e-5, 1e-4)
    check_solution(g, r.eigenvalues, to_np(r.H), k, normalized, tol, G.sigma, lam_ref, H_ref, rtol, ang, gap)


@pytest.mark.parametrize("normalized", [False, True])
def test_plain_sc_h1_on_the_same_kernels(normalized):
    # plain spectral clustering = the fair problem with one group (F has no
    # columns, P = I, L^sigma = L); the oracle's h = 1 case is the textbook
    # eigenproblem (pinned in test_oracle_pins); lambda_1 = 0 is the trivial pair
    import dataclasses

    sf = lib()
    g0 = workload("msbm-2k-h2")
    g = dataclasses.replace(g0, groups=np.zeros(g0.n, dtype=np.int32), h=1)
    k, tol = 5, 1e-10
    lam_ref, H_ref = oracle.fair_eigs_dense(g.to_scipy(), g.groups, 1, k + 1, normalized)
    assert abs(lam_ref[0]) <= 1e-10 * lam_ref[1]
    G = sf.Graph.from_msbm(g, normalized)
    r = G.eigs(k, tol=tol, precision="fp64")
    log(f"plain SC normalized={normalized}: info {r.info}")
    gap = (lam_ref[k] - lam_ref[k - 1]) / G.sigma
    check_solution(g, r.eigenvalues, to_np(r.H), k, normalized, tol, G.sigma, lam_ref, H_ref, 1e-8, 1e-6, gap)
    rm = G.eigs(k, tol=1e-6, precision="mixed")
    check_solution(g, rm.eigenvalues, to_np(rm.H), k, normalized, 1e-6, G.sigma, lam_ref, H_ref, 1e-5, 1e-4, gap)


def test_complete_graph_breakdown_is_repaired():
    # K_n has only the eigenvalues 0 and n (and sigma after deflation): the
    # Krylov space becomes invariant after a few blocks and must be repaired
    sf = lib()
    n, h = 64, 4
    rows = np.repeat(np.arange(n), n - 1)
    cols = np.concatenate([np.delete(np.arange(n), i) for i in range(n)])
    rowptr = np.arange(0, n * (n - 1) + 1, n - 1, dtype=np.int32)
    G = sf.Graph(rowptr, cols.astype(np.int32), np.ones(n * (n - 1)), (np.arange(n) % h).astype(np.int32), h, False)
    with pytest.warns(RuntimeWarning):
        r = G.eigs(6, tol=1e-10)
    log(f"  info {r.info}")
    # theta_6 = theta_7 = n: k splits the multiple eigenvalue n
    assert r.status == sf.E_DEGENERATE
    assert abs(r.eigenvalues[0]) < 1e-8 * n
    assert np.allclose(r.eigenvalues[1:], n, rtol=1e-9)


def test_disjoint_fair_cliques_zero_eigenspace():
    # k disjoint fair cliques: eigenvalue 0 with multiplicity k, eigenspace
    # spanned by the clique indicators (the eigenspace-mixing case)
    sf = lib()
    k, per = 4, 40
    n = k * per
    blocks = []
    for c in range(k):
        for i in range(per):
            for j in range(per):
                if i != j:
                    blocks.append((c * per + i, c * per + j))
    e = np.array(blocks)
    W = sp.csr_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    W.sort_indices()
    groups = (np.arange(n) % 2).astype(np.int32)
    for normalized in (False, True):
        G = sf.Graph(W.indptr.astype(np.int32), W.indices.astype(np.int32), W.data, groups, 2, normalized)
        r = G.eigs(k, tol=1e-10)
        assert np.all(np.abs(r.eigenvalues) < 1e-8 * G.sigma)
        ind = np.kron(np.eye(k), np.ones((per, 1)))
        d = np.asarray(W.sum(1)).ravel() if normalized else None
        assert oracle.max_principal_angle(to_np(r.H), ind, d) < 1e-6


def _fair_cliques(nc, per):
    n = nc * per
    e = np.array([(c * per + i, c * per + j) for c in range(nc) for i in range(per) for j in range(per) if i != j])
    W = sp.csr_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    W.sort_indices()
    return W, (np.arange(n) % 2).astype(np.int32)


@pytest.mark.parametrize("normalized", [False, True])
def test_many_equal_eigenvalues_across_restarts(normalized):
    # 24 disjoint fair cliques of 12: the fair eigenvalue 0 has multiplicity 24
    # and every clique contributes the same nonzero eigenvalues, so Ritz
    # values coincide in large clusters; a restart may then keep more vectors
    # than the rule's count (the cluster is not split), which the solver
    # learns only from the Rayleigh-Ritz record.  k = 24 takes the whole zero
    # eigenspace.
    sf = lib()
    nc, per = 24, 12
    W, groups = _fair_cliques(nc, per)
    G = sf.Graph(W.indptr.astype(np.int32), W.indices.astype(np.int32), W.data, groups, 2, normalized)
    r = G.eigs(nc, tol=1e-10, block_width=8, max_basis=96)
    log(f"  info {r.info}")
    assert r.status == sf.OK
    assert 0 <= r.info["restarts_unpredicted"] < r.info["restarts"]
    assert np.all(np.abs(r.eigenvalues) < 1e-8 * G.sigma)
    H = to_np(r.H)
    d = np.asarray(W.sum(1)).ravel()
    M = H.T @ (d[:, None] * H) if normalized else H.T @ H
    assert np.abs(M - np.eye(nc)).max() < 1e-9
    ind = np.kron(np.eye(nc), np.ones((per, 1)))
    assert oracle.max_principal_angle(H, ind, d if normalized else None) < 1e-6
    res = oracle.residual_norms(W, groups, 2, normalized, r.eigenvalues, H)
    assert res.max() <= 1e-10 * G.sigma + 2e-12 * G.sigma


@pytest.mark.parametrize("normalized", [False, True])
def test_k_splitting_a_multiple_eigenvalue_is_flagged(normalized):
    # 4 disjoint fair cliques: the fair eigenvalue 0 has multiplicity 4.
    # k = 2 splits it, so theta_2 = theta_3 and the 2-dimensional subspace is
    # not determined: E_DEGENERATE with the outputs written (two orthonormal
    # vectors of the zero eigenspace).  k = 4 takes the whole eigenspace: OK.
    sf = lib()
    W, groups = _fair_cliques(4, 40)
    n = W.shape[0]
    G = sf.Graph(W.indptr.astype(np.int32), W.indices.astype(np.int32), W.data, groups, 2, normalized)
    with pytest.warns(RuntimeWarning):
        r = G.eigs(2, tol=1e-10)
    log(f"  k=2 info {r.info}")
    assert r.status == sf.E_DEGENERATE and r.info["degenerate"] == 1
    assert r.info["gap_ratio"] <= 100 * 1e-10
    assert np.all(np.abs(r.eigenvalues) < 1e-8 * G.sigma)
    H = to_np(r.H)
    d = np.asarray(W.sum(1)).ravel()
    M = H.T @ (d[:, None] * H) if normalized else H.T @ H
    assert np.abs(M - np.eye(2)).max() < 1e-9
    ind = np.kron(np.eye(4), np.ones((40, 1)))
    Qi = np.linalg.qr(ind)[0]
    assert np.abs(H - Qi @ (Qi.T @ H)).max() < 1e-8 * np.abs(H).max()  # inside the zero eigenspace
    with pytest.raises(sf.SfairscError) as e:
        G.eigs(2, tol=1e-10, raise_degenerate=True)
    assert e.value.code == sf.E_DEGENERATE
    r4 = G.eigs(4, tol=1e-10)
    assert r4.status == sf.OK and r4.info["degenerate"] == 0 and r4.info["gap_ratio"] > 0.1


def test_degenerate_status_in_a_batch():
    sf = lib()
    W, groups = _fair_cliques(4, 40)
    Gs = [sf.Graph(W.indptr.astype(np.int32), W.indices.astype(np.int32), W.data, groups, 2, False) for _ in range(2)]
    g2 = workload("msbm-2k-h2")
    Gs.append(sf.Graph.from_msbm(g2, False))
    with pytest.warns(RuntimeWarning):
        rs = sf.eigs_batched(Gs, [2, 4, 5], tol=1e-8, precision="fp64")
    assert [r.status for r in rs] == [sf.E_DEGENERATE, sf.OK, sf.OK], [r.info for r in rs]


def test_rank_deficient_start_block_is_reported():
    # a warm start whose two columns coincide: the start block's Cholesky-QR
    # fails; the solver learns it from the first Rayleigh-Ritz record (every
    # kernel in between skips its work) and reports E_ARG
    sf = lib()
    g = random_sparse_graph(1200, 10, seed=31, h=3)
    G = sf.Graph.from_msbm(g, False)
    v = torch.from_numpy(np.random.default_rng(4).standard_normal((g.n, 1)))
    with pytest.raises(sf.SfairscError) as e:
        G.eigs(4, tol=1e-8, x0=torch.cat([v, v], dim=1))
    assert e.value.code == sf.E_ARG and "rank deficient" in str(e.value)
    # the handle is still good: a valid warm start and a plain solve
    r = G.eigs(4, tol=1e-8, x0=torch.cat([v, 2 * v + 1], dim=1))
    r2 = G.eigs(4, tol=1e-8)
    assert np.abs(r.eigenvalues - r2.eigenvalues).max() <= 1e-8 * G.sigma


def test_not_converged_returns_partial_result():
    sf = lib()
    g = workload("msbm-2k-h2")
    G = sf.Graph.from_msbm(g, False)
    r = G.eigs(5, tol=1e-15, max_restarts=1, raise_not_converged=False)
    assert r.status == sf.E_NOT_CONVERGED
    assert r.info["restarts"] == 1
    assert np.all(np.isfinite(r.eigenvalues)) and torch.isfinite(r.H).all()


def test_bitwise_repeatable_and_warm_start():
    sf = lib()
    g = workload("msbm-2k-h2")
    G = sf.Graph.from_msbm(g, True)
    a = G.eigs(5, tol=1e-10)
    b = G.eigs(5, tol=1e-10)
    assert np.array_equal(a.eigenvalues, b.eigenvalues)
    assert torch.equal(a.H, b.H)
    # warm start from the (back-transformed) solution: X = D^{1/2} H
    d = torch.from_numpy(oracle.degrees(g.to_scipy())).to(a.H.device)
    x0 = (a.H * d.sqrt()[:, None]).contiguous()
    c = G.eigs(5, tol=1e-10, x0=x0, block_width=8)
    assert c.info["restarts"] <= a.info["restarts"]
    assert eig_parity(c.eigenvalues, a.eigenvalues, 1e-8) <= 1e-8


def test_msbm_50k_normalized_fp64_and_mixed():
    # the n = 50,000 normalized workload against stored oracle eigenvalues
    # (tests/golden/make_golden.py) and the oracle's residuals
    sf = lib()
    gold = read_golden("msbm50k_normalized_eigs.txt")
    lam_ref = np.array([float(x) for x in gold["eigenvalues"]])
    g = workload("msbm-50k-h5-normalized")
    G = sf.Graph.from_msbm(g, True)
    k, tol = 10, 1e-8
    # the oracle's eigenvectors (implicit nullspace + ARPACK, Tier B) for the
    # subspace angle; relative gap (lambda_11 - lambda_10) / sigma ~ 0.08
    lam_b, H_b = oracle.fair_eigs_implicit(g.to_scipy(), g.groups, g.h, k + 1, True, tol=1e-13)
    assert eig_parity(lam_b[:k], lam_ref[:k], 1e-11) <= 1e-11
    gap = (lam_b[k] - lam_b[k - 1]) / G.sigma
    for prec, rtol, atol_angle in (("fp64", 1e-8, 1e-6), ("mixed", 1e-5, 1e-4)):
        log(f"msbm-50k {prec}")
        r = G.eigs(k, tol=tol, precision=prec)
        log(f"  info {r.info}")
        check_solution(g, r.eigenvalues, to_np(r.H), k, True, tol, G.sigma, lam_ref, H_b, rtol, atol_angle, gap)


def test_kernel_timing_mode_reports_the_phases():
    # time_kernels: GPU event time of the operator (which contains the sparse
    # product), the orthogonalisation and the restart rotation; zero otherwise
    sf = lib()
    g = random_sparse_graph(3000, 20, seed=91, h=3)
    G = sf.Graph.from_msbm(g, True)
    r = G.eigs(6, tol=1e-9, precision="fp64", block_width=8, max_basis=32, time_kernels=True)
    i = r.info
    log(f"timing info {i}")
    assert i["operator_ms"] > 0 and i["ortho_ms"] > 0
    assert (i["restart_ms"] > 0) == (i["restarts"] > 0)
    assert i["operator_ms"] >= sum(i["spmm_ms"]) > 0
    r0 = G.eigs(6, tol=1e-9, precision="fp64", block_width=8, max_basis=32)
    assert r0.info["operator_ms"] == 0 and r0.info["ortho_ms"] == 0 and r0.info["restart_ms"] == 0
    assert np.allclose(r0.eigenvalues, r.eigenvalues, rtol=1e-10)
