"""Parity of the GPU k-means (sfairsc_labels) with the oracle's (GPU).

Both sides implement the same specification (k-means++ with SplitMix64
uniforms, Lloyd with lowest-index ties, best of restarts, first-appearance
numbering).  On the same input rows the labels must be identical; the
inertia agrees to rounding (different summation order).
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_common import lib, log, to_np
from sfairsc_inputs import random_sparse_graph, workload

pytestmark = pytest.mark.gpu


def _graph_for(sf, n):
    # any handle of the right size: labels only use n
    g = random_sparse_graph(n, 4, seed=n, h=2)
    return sf.Graph.from_msbm(g, False)


@pytest.mark.parametrize("normalized", [False, True])
def test_labels_match_oracle_on_fair_embedding(normalized):
    sf = lib()
    g = workload("msbm-2k-h2")
    _, H = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, 5, normalized)
    G = sf.Graph.from_msbm(g, normalized)
    lab_gpu, inertia_gpu = G.labels(torch.from_numpy(H), 5, n_restarts=10, seed=0)
    lab_ref, inertia_ref = oracle.kmeans(H, 5, 10, 0)
    assert np.array_equal(to_np(lab_gpu), lab_ref)
    assert inertia_gpu == pytest.approx(inertia_ref, rel=1e-10)
    assert oracle.error_rate(lab_ref, g.clusters) == 0.0


@pytest.mark.parametrize("seed", [0, 1, 7])
@pytest.mark.parametrize("shape", [(3001, 4, 6), (517, 3, 2), (12000, 10, 10)])
def test_labels_match_oracle_on_overlapping_blobs(seed, shape):
    # overlapping clusters: many Lloyd iterations and seeding decisions
    sf = lib()
    n, K, dim = shape
    rng = np.random.default_rng(seed)
    centers = rng.standard_normal((K, dim))
    X = centers[rng.integers(0, K, n)] + 0.6 * rng.standard_normal((n, dim))
    G = _graph_for(sf, n)
    lab_gpu, inertia_gpu = G.labels(torch.from_numpy(X), K, n_restarts=4, seed=seed)
    lab_ref, inertia_ref = oracle.kmeans(X, K, 4, seed)
    log(f"blobs {shape} seed {seed}: inertia {inertia_gpu} vs {inertia_ref}")
    assert inertia_gpu == pytest.approx(inertia_ref, rel=1e-10)
    assert np.array_equal(to_np(lab_gpu), lab_ref)


@pytest.mark.parametrize("n,K,dim,R", [(1500, 64, 20, 3), (900, 12, 40, 260), (700, 5, 3, 257)])
def test_labels_edge_shapes(n, K, dim, R):
    # the most clusters (64: every bit of the first-appearance mask), rows
    # of 20 and 40 values (the wider register layouts of the assignment)
    # and more restarts than the best-restart workgroup has threads
    sf = lib()
    rng = np.random.default_rng(5)
    X = (4.0 * rng.standard_normal((K, dim)))[rng.integers(0, K, n)] + 0.6 * rng.standard_normal((n, dim))
    G = _graph_for(sf, n)
    lab_gpu, inertia_gpu = G.labels(torch.from_numpy(X), K, n_restarts=R, seed=5)
    lab_ref, inertia_ref = oracle.kmeans(X, K, R, 5)
    log(f"edge shape n={n} K={K} dim={dim} R={R}: inertia {inertia_gpu} vs {inertia_ref}")
    assert inertia_gpu == pytest.approx(inertia_ref, rel=1e-10)
    assert np.array_equal(to_np(lab_gpu), lab_ref)


def test_labels_rotation_invariant_and_bruteforce_small():
    sf = lib()
    rng = np.random.default_rng(3)
    X = np.concatenate([c + 0.05 * rng.standard_normal((50, 4)) for c in 3 * rng.standard_normal((4, 4))])
    G = _graph_for(sf, X.shape[0])
    a, _ = G.labels(torch.from_numpy(X), 4, 5, 0)
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    b, _ = G.labels(torch.from_numpy(X @ Q), 4, 5, 0)
    assert torch.equal(a, b)
    assert oracle.same_partition(to_np(a), np.repeat(np.arange(4), 50))


def test_labels_degenerate_points():
    sf = lib()
    X = np.ones((300, 2))
    X[::7] += 1.0
    G = _graph_for(sf, 300)
    lab, inertia = G.labels(torch.from_numpy(X), 3, 2, 0)
    lab_ref, inertia_ref = oracle.kmeans(X, 3, 2, 0)
    assert np.array_equal(to_np(lab), lab_ref)
    assert inertia == pytest.approx(inertia_ref, abs=1e-12)
