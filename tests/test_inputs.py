"""The seeded m-SBM generator (paper, Appendix B.1) — CPU only."""

import numpy as np
import pytest

from conftest import read_golden
from sfairsc_inputs import msbm_from_blocks, relabel, workload, random_sparse_graph
from sfairsc_inputs.msbm import batched_specs, batched_graph, fair_block_sizes, scale_for_degree


def _check_csr(g):
    n = g.n
    assert g.rowptr.dtype == np.int32 and g.col.dtype == np.int32
    assert g.rowptr[0] == 0 and g.rowptr[-1] == g.col.size == g.val.size
    rows = g.row_index()
    assert np.all(rows != g.col), "self-loop"
    # sorted, no duplicates within rows
    key = rows.astype(np.int64) * n + g.col
    assert np.all(np.diff(key) > 0)
    W = g.to_scipy()
    assert abs(W - W.T).max() == 0, "not symmetric"
    assert np.all(g.val > 0)


def test_example_b2_layout():
    gold = read_golden("example_b2_msbm.txt")
    u = np.array(list(map(int, gold["u"]))).reshape(3, 2)
    # the paper's a, b, c, d = 0.6, 0.4, 0.2, 0.1 with b = different cluster /
    # same group and c = same cluster / different group
    g = msbm_from_blocks(u, (0.6, 0.2, 0.4, 0.1), seed=7, weights=("alpha_beta", 3.0, 1.0))
    assert g.n == 10
    g1 = np.array(list(map(int, gold["g1"])))
    g2 = np.array(list(map(int, gold["g2"])))
    assert np.array_equal((g.groups == 0).astype(int), g1)
    assert np.array_equal((g.groups == 1).astype(int), g2)
    for c in range(3):
        col = np.array(list(map(int, gold[f"H_col{c + 1}"])))
        assert np.array_equal((g.clusters == c).astype(int), col)
    _check_csr(g)
    # weights alpha within clusters, beta between (eq. msbm-bernoulli)
    rows = g.row_index()
    same = g.clusters[rows] == g.clusters[g.col]
    assert np.all(g.val[same] == 3.0) and np.all(g.val[~same] == 1.0)


def test_planted_clustering_is_exactly_fair():
    g = workload("msbm-2k-h2")
    _check_csr(g)
    n = g.n
    for c in range(g.k):
        cnt = np.bincount(g.groups[g.clusters == c], minlength=g.h)
        tot = np.bincount(g.groups, minlength=g.h)
        # eq. fair: |V_s cap C_l| / |C_l| = |V_s| / |V|, in integers
        assert np.all(cnt * n == tot * cnt.sum())


def test_block_densities_match_probabilities():
    u = fair_block_sizes([300] * 4, [1, 2])
    probs = (0.3, 0.2, 0.08, 0.03)
    g = msbm_from_blocks(u, probs, seed=11)
    rows = g.row_index()
    up = rows < g.col
    i, j = rows[up], g.col[up]
    same_c = g.clusters[i] == g.clusters[j]
    same_g = g.groups[i] == g.groups[j]
    n = g.n
    cl = g.clusters
    gr = g.groups
    # count candidate pairs of each relation
    pairs = {}
    for sc in (True, False):
        for sg in (True, False):
            tot = 0
            for a in range(4):
                for b in range(2):
                    na = int(((cl == a) & (gr == b)).sum())
                    for a2 in range(4):
                        for b2 in range(2):
                            if ((a == a2) != sc) or ((b == b2) != sg):
                                continue
                            nb = int(((cl == a2) & (gr == b2)).sum())
                            tot += na * (nb - 1) if (a == a2 and b == b2) else na * nb
            pairs[(sc, sg)] = tot // 2
    p = {(True, True): probs[0], (True, False): probs[1], (False, True): probs[2], (False, False): probs[3]}
    for key, npairs in pairs.items():
        m = int(np.count_nonzero((same_c == key[0]) & (same_g == key[1])))
        mean = npairs * p[key]
        sd = np.sqrt(npairs * p[key] * (1 - p[key]))
        assert abs(m - mean) < 5 * sd + 1, (key, m, mean, sd)
    assert n == 1200


def test_isolated_vertices_are_repaired():
    u = np.array([[200, 200]])
    g = msbm_from_blocks(u, (0.002, 0.002, 0.0, 0.0), seed=3)
    deg = np.diff(g.rowptr)
    assert deg.min() >= 1
    assert g.n_repaired > 0
    _check_csr(g)


def test_relabel_is_an_isomorphism():
    g = workload("msbm-2k-h2")
    r = relabel(g, 9)
    _check_csr(r)
    assert r.nnz == g.nnz
    assert np.array_equal(np.sort(np.diff(r.rowptr)), np.sort(np.diff(g.rowptr)))
    assert np.array_equal(np.bincount(r.groups), np.bincount(g.groups))
    # edges map onto edges: total weight between (cluster, group) classes preserved
    def cls_weights(x):
        rows = x.row_index()
        key = (x.clusters[rows] * 10 + x.groups[rows]) * 100 + x.clusters[x.col] * 10 + x.groups[x.col]
        return np.bincount(key, weights=x.val, minlength=10000)
    assert np.array_equal(cls_weights(r), cls_weights(g))


def test_generator_is_deterministic():
    a = workload("msbm-500-h4-grad")
    b = workload("msbm-500-h4-grad")
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert a.val.dtype == np.float32
    assert 0.5 <= a.val.min() and a.val.max() <= 1.5


def test_degree_scaling():
    u = fair_block_sizes([20000] * 10, [1] * 4)
    probs = scale_for_degree(u, (4.0, 3.0, 1.0, 0.5), 40.0)
    assert probs[0] / probs[3] == pytest.approx(8.0)


def test_random_sparse_graph_and_batched_specs():
    g = random_sparse_graph(500, 12, seed=1, h=3)
    _check_csr(g)
    assert set(np.unique(g.groups)) == {0, 1, 2}
    specs = batched_specs(256)
    ns = np.array([s["n"] for s in specs])
    assert ns.min() >= 1000 and ns.max() <= 50000
    assert {s["k"] for s in specs} <= set(range(2, 11))
    assert {s["h"] for s in specs} <= set(range(2, 7))
    small = min(specs, key=lambda s: s["n"])
    gb = batched_graph(small)
    _check_csr(gb)
    assert gb.n == small["n"]
