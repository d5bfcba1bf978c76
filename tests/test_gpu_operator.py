"""Parity of the operator kernels against the oracle (GPU).

The deflated operator Y = L^sigma X (eq. asigma, applied by the matvec
formula of Section 3.4) and the bare sparse product are compared element by
element with the FP64 oracle on seeded graphs that span many row tiles and a
ragged tail, for several block widths (padded and unpadded) and both
variants.

Tolerances.  Row i of L X' is d_i x'_i - sum_j w_ij x'_j: at most deg_i + 1
terms whose magnitudes add up to at most 2 d_i max|X| <= sigma max|X|
(sigma = ||L||_1; the normalized case is the same with L_n).  Recursive
summation in precision u therefore errs by at most (deg_max + 1) u sigma
max|X|, and rounding X' to float adds u sigma max|X|.  Mixed precision
(u = 2^-24) is checked against 2 (deg_max + 2) 2^-24 sigma max|X|.  FP64
(u = 2^-53) adds the projection's group sums over up to n rows, blocked
into per-thread runs of n / 2048 terms; 1e-12 sigma max|X| bounds both for
the graphs here (deg_max <= 164, n <= 50,000).
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_common import lib, log, to_np
from sfairsc_inputs import random_sparse_graph, workload

pytestmark = pytest.mark.gpu

CASES = [
    # (graph builder, h label, normalized)
    ("er-1031-h3", lambda: random_sparse_graph(1031, 17, seed=1, h=3), False),
    ("er-1031-h3", lambda: random_sparse_graph(1031, 17, seed=1, h=3), True),
    ("er-777-h1", lambda: random_sparse_graph(777, 9, seed=2, h=1), False),
    ("msbm-2k-h2", lambda: workload("msbm-2k-h2"), False),
    ("msbm-2k-h2", lambda: workload("msbm-2k-h2"), True),
    ("msbm-500-h4", lambda: workload("msbm-500-h4-grad"), False),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("b", [1, 3, 4, 8, 13, 16, 32])
def test_apply_operator_fp64_and_mixed(case, b):
    sf = lib()
    name, build, normalized = CASES[case]
    log(f"operator {name} normalized={normalized} b={b}")
    g = build()
    W = g.to_scipy()
    G = sf.Graph.from_msbm(g, normalized)
    sigma = G.sigma
    assert sigma == pytest.approx(oracle.shift_sigma(W, normalized), rel=1e-13)
    rng = np.random.default_rng(b + 10 * case)
    X = rng.standard_normal((g.n, b))
    ref = oracle.apply_deflated_operator(W, g.groups, g.h, normalized, sigma, X)
    Y = to_np(G.apply_operator(torch.from_numpy(X), "fp64"))
    scale = sigma * np.abs(X).max()
    assert np.abs(Y - ref).max() <= 1e-12 * scale
    Ym = to_np(G.apply_operator(torch.from_numpy(X), "mixed"))
    assert np.abs(Ym - ref).max() <= mixed_tol(g) * scale


SETUP_CASES = [
    # (mean degree, h, value dtype): the set-up passes give a CSR row 8, 16,
    # 32 or 64 lanes by mean degree (8 below 64, 64 from 256 on); h up to the
    # maximum of 32 groups
    (4, 2, np.float64),
    (30, 32, np.float32),
    (90, 5, np.float64),
    (150, 7, np.float32),
    (300, 3, np.float64),
]


def _with_hub(g, every):
    # vertex 0 joined to every `every`-th vertex: one row far longer than a
    # wavefront, whatever the lanes per row
    import scipy.sparse as sp

    W = g.to_scipy(g.val.dtype).tolil()
    for j in range(every, g.n, every):
        W[0, j] = W[j, 0] = 0.75
    W = sp.csr_matrix(W)
    W.sort_indices()
    return W


@pytest.mark.parametrize("case", range(len(SETUP_CASES)))
@pytest.mark.parametrize("normalized", [False, True])
def test_graph_setup_against_the_oracle(case, normalized):
    sf = lib()
    deg, h, dt = SETUP_CASES[case]
    log(f"set-up mean degree {deg} h={h} {np.dtype(dt).name} normalized={normalized}")
    g = random_sparse_graph(3001, deg, seed=11 + case, h=h, val_dtype=dt)
    W = _with_hub(g, 3)
    val = W.data.astype(dt)
    G = sf.Graph(W.indptr.astype(np.int32), W.indices.astype(np.int32), val, g.groups, h, normalized)
    W64 = W.astype(np.float64)
    d = oracle.degrees(W64)
    st = G.stats()
    assert st["sigma"] == pytest.approx(oracle.shift_sigma(W64, normalized), rel=1e-13)
    assert st["min_degree"] == pytest.approx(d.min(), rel=1e-13)
    assert st["max_degree"] == pytest.approx(d.max(), rel=1e-13)
    assert st["nnz"] == W.nnz and st["h"] == h
    # the values, the diagonal and the closed form of (C^T C)^{-1} all enter
    # the operator
    X = np.random.default_rng(case).standard_normal((g.n, 4))
    ref = oracle.apply_deflated_operator(W64, g.groups, h, normalized, G.sigma, X)
    Y = to_np(G.apply_operator(torch.from_numpy(X), "fp64"))
    assert np.abs(Y - ref).max() <= 1e-12 * G.sigma * np.abs(X).max()
    G.close()


def mixed_tol(g):
    deg_max = int(np.diff(g.rowptr).max())
    return 2.0 * (deg_max + 2) * 2.0**-24


@pytest.mark.parametrize("normalized", [False, True])
@pytest.mark.parametrize("b", [2, 8, 16, 32])
def test_spmm_matches_sparse_product(normalized, b):
    sf = lib()
    g = workload("msbm-2k-h2")
    W = g.to_scipy()
    A = oracle.normalized_laplacian(W) if normalized else oracle.laplacian(W)
    G = sf.Graph.from_msbm(g, normalized)
    X = np.random.default_rng(b).standard_normal((g.n, b))
    T = to_np(G.spmm(torch.from_numpy(X), "fp64"))
    ref = A @ X
    s = G.sigma * np.abs(X).max()
    assert np.abs(T - ref).max() <= 1e-12 * s
    T32 = to_np(G.spmm(torch.from_numpy(X.astype(np.float32)), "mixed")).astype(np.float64)
    ref32 = A @ X.astype(np.float32).astype(np.float64)
    assert np.abs(T32 - ref32).max() <= mixed_tol(g) * s


def test_constraint_range_is_the_sigma_eigenspace():
    # L^sigma C = sigma C (Props. 3.1-3.2): the range of C is shifted to sigma
    sf = lib()
    g = random_sparse_graph(1500, 11, seed=3, h=5)
    for normalized in (False, True):
        G = sf.Graph.from_msbm(g, normalized)
        C = oracle.constraint_matrix(g.to_scipy(), g.groups, 5, normalized)
        Y = to_np(G.apply_operator(torch.from_numpy(C), "fp64"))
        assert np.abs(Y - G.sigma * C).max() <= 1e-12 * G.sigma * np.abs(C).max()


def test_operator_full_size_normalized_50k():
    # the n = 50,000 normalized workload, one block of 16, all rows checked
    sf = lib()
    g = workload("msbm-50k-h5-normalized")
    W = g.to_scipy()
    G = sf.Graph.from_msbm(g, True)
    X = np.random.default_rng(5).standard_normal((g.n, 16))
    ref = oracle.apply_deflated_operator(W, g.groups, g.h, True, G.sigma, X)
    s = G.sigma * np.abs(X).max()
    Y = to_np(G.apply_operator(torch.from_numpy(X), "fp64"))
    assert np.abs(Y - ref).max() <= 1e-12 * s
    Ym = to_np(G.apply_operator(torch.from_numpy(X), "mixed"))
    assert np.abs(Ym - ref).max() <= mixed_tol(g) * s


def test_operator_is_deterministic():
    sf = lib()
    g = workload("msbm-2k-h2")
    G = sf.Graph.from_msbm(g, True)
    X = torch.from_numpy(np.random.default_rng(0).standard_normal((g.n, 16)))
    a = G.apply_operator(X, "mixed")
    b = G.apply_operator(X, "mixed")
    assert torch.equal(a, b)
