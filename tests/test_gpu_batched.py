"""Parity of the batched persistent solve (sfairsc_eigs_batched) and of the
autotuner's table (GPU).

Every graph of a batch must meet the single-graph bars against the FP64
oracle: eigenvalues relative 1e-8 (FP64) / 1e-5 (float sparse products),
largest principal angle 1e-6 / 1e-4 when the relative gap exceeds 100 tol,
F^T H = 0, orthonormality, and the oracle's residual of each pair below the
tolerance.  Graphs are modified SBMs of uneven size with the batched
workload's recipe (probability ratios 4:3:1:0.5, equal groups).
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_common import eig_parity, lib, log, to_np
from sfairsc_inputs.msbm import batched_graph, batched_specs

pytestmark = pytest.mark.gpu

SMALL_SPECS = [
    dict(n=1000, k=2, h=2, avg_degree=12.0, seed=901),
    dict(n=1500, k=5, h=3, avg_degree=40.0, seed=902),
    dict(n=2200, k=10, h=6, avg_degree=75.0, seed=903),
    dict(n=1300, k=7, h=4, avg_degree=25.0, seed=904),
    dict(n=1800, k=3, h=5, avg_degree=60.0, seed=905),
    dict(n=2500, k=9, h=2, avg_degree=18.0, seed=906),
]


def _graphs(specs, normalized_every=2):
    out = []
    for i, s in enumerate(specs):
        g = batched_graph(s)
        out.append((g, s["k"], normalized_every > 0 and i % normalized_every == 1))
    return out


def _refs(items):
    refs = []
    for g, k, norm in items:
        lam, H = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, k + 1, norm)
        refs.append((lam, H))
    return refs


def _check(g, k, norm, r, sigma, tol, lam_ref, H_ref, rtol, atol_angle):
    W = g.to_scipy()
    d = oracle.degrees(W)
    lam = r.eigenvalues
    H = to_np(r.H)
    assert np.all(np.diff(lam) >= -1e-12 * sigma)
    F = oracle.fairness_matrix(g.groups, g.h)
    assert np.abs(F.T @ H).max() <= 1e-10 * np.sqrt(g.n) * np.abs(H).max()
    M = H.T @ (d[:, None] * H) if norm else H.T @ H
    assert np.abs(M - np.eye(k)).max() <= 1e-9
    # returned pairs meet tol on the library's FP64 residual, which for
    # vectors in null(C^T) equals the oracle's: only rounding separates them
    res = oracle.residual_norms(W, g.groups, g.h, norm, lam, H)
    assert res.max() <= tol * sigma + 2e-12 * sigma, res.max() / sigma
    err = eig_parity(lam, lam_ref[:k], rtol)
    assert err <= rtol, err
    gap = (lam_ref[k] - lam_ref[k - 1]) / sigma
    ang = None
    if gap > 100 * tol:
        ang = oracle.max_principal_angle(H, H_ref[:, :k], d if norm else None)
        assert ang <= atol_angle, ang
    return err, ang


@pytest.fixture(scope="module")
def small():
    items = _graphs(SMALL_SPECS)
    return items, _refs(items)


def _handles(sf, items):
    return [sf.Graph.from_msbm(g, norm) for g, _, norm in items]


@pytest.mark.parametrize("precision,tol,rtol,angle", [("fp64", 1e-10, 1e-8, 1e-6), ("mixed", 1e-6, 1e-5, 1e-4)])
def test_batched_small_parity(small, precision, tol, rtol, angle):
    sf = lib()
    items, refs = small
    Gs = _handles(sf, items)
    log(f"batched {len(Gs)} graphs {precision} tol {tol}")
    rs = sf.eigs_batched(Gs, [k for _, k, _ in items], tol=tol, precision=precision)
    for (g, k, norm), G, r, (lam_ref, H_ref) in zip(items, Gs, rs, refs):
        log(f"  n={g.n} k={k} h={g.h} norm={norm} info={r.info}")
        assert r.info["path"] == 0 and r.info["batch_status"] == 0, r.info
        assert r.info["double_spmm"] == (1 if precision == "fp64" else 0)
        err, ang = _check(g, k, norm, r, G.sigma, tol, lam_ref, H_ref, rtol, angle)
        log(f"    eig rel err {err:.2e} angle {ang}")


@pytest.mark.parametrize("bw", [4, 8, 16])
def test_batched_forced_block_width(small, bw):
    sf = lib()
    items, refs = small
    Gs = _handles(sf, items)
    tol = 1e-10
    ks = [k for _, k, _ in items]
    log(f"batched forced b={bw}")
    rs = sf.eigs_batched(Gs, ks, tol=tol, precision="fp64", block_width=bw)
    for (g, k, norm), G, r, (lam_ref, H_ref) in zip(items, Gs, rs, refs):
        assert r.info["block_width"] == bw
        if r.info["path"] == 0:
            assert r.info["batch_status"] == 0, r.info
        _check(g, k, norm, r, G.sigma, tol, lam_ref, H_ref, 1e-8, 1e-6)


def test_batched_repeatable_and_matches_single(small):
    sf = lib()
    items, _ = small
    Gs = _handles(sf, items)
    ks = [k for _, k, _ in items]
    r1 = sf.eigs_batched(Gs, ks, tol=1e-10, precision="fp64", seed=7)
    r2 = sf.eigs_batched(Gs, ks, tol=1e-10, precision="fp64", seed=7)
    for a, b, G, k in zip(r1, r2, Gs, ks):
        assert np.array_equal(a.eigenvalues, b.eigenvalues)
        assert torch.equal(a.H, b.H)
        s = G.eigs(k, tol=1e-10, precision="fp64")
        assert eig_parity(a.eigenvalues, s.eigenvalues, 1e-9) <= 1e-9


def test_batched_fallback_paths():
    # a graph too small for the launch's basis and a k beyond its limit are
    # solved by the single-graph solver; results meet the same bars
    sf = lib()
    items = _graphs([dict(n=40, k=3, h=2, avg_degree=8.0, seed=911),
                     dict(n=1600, k=50, h=3, avg_degree=30.0, seed=912),
                     dict(n=1400, k=4, h=2, avg_degree=30.0, seed=913)], normalized_every=0)
    refs = _refs(items)
    Gs = _handles(sf, items)
    rs = sf.eigs_batched(Gs, [k for _, k, _ in items], tol=1e-9, precision="fp64")
    paths = [r.info["path"] for r in rs]
    log(f"  paths {paths}")
    assert paths == [1, 1, 0]
    for (g, k, norm), G, r, (lam_ref, H_ref) in zip(items, Gs, rs, refs):
        _check(g, k, norm, r, G.sigma, 1e-9, lam_ref, H_ref, 1e-8, 1e-6)


def test_batched_argument_errors(small):
    sf = lib()
    items, _ = small
    Gs = _handles(sf, items[:2])
    with pytest.raises(sf.SfairscError):
        sf.eigs_batched(Gs, [2, 5], tol=1e-8, precision="fp64", block_width=32)
    with pytest.raises(sf.SfairscError):
        sf.eigs_batched(Gs, [2, 5], tol=1e-8, precision="fp64", block_width=8, max_basis=12)
    with pytest.raises(sf.SfairscError):
        sf.eigs_batched(Gs, [0, 5], tol=1e-8)
    with pytest.raises(sf.SfairscError):
        sf.eigs_batched(Gs, [2, 5], tol=-1.0)


def test_autotune_fills_the_table(small, tmp_path):
    sf = lib()
    items, refs = small
    Gs = _handles(sf, items)
    ks = [k for _, k, _ in items]
    sf.tuning_clear()
    try:
        size = sf.autotune(Gs, ks, tol=1e-6, precision="mixed", per_bucket=1)
        log(f"  tuning entries {size}")
        assert size >= 1
        hits = [sf.tuning_lookup(g.n, g.nnz, k, "mixed", norm, 1e-6)[3] for g, k, norm in items]
        assert all(hits)
        rs = sf.eigs_batched(Gs, ks, tol=1e-6, precision="mixed")
        for (g, k, norm), G, r, (lam_ref, H_ref) in zip(items, Gs, rs, refs):
            assert r.info["from_table"] == 1 and r.info["path"] == 0, r.info
            _check(g, k, norm, r, G.sigma, 1e-6, lam_ref, H_ref, 1e-5, 1e-4)
        path = tmp_path / "table.json"
        sf.tuning_save(str(path))
        sf.tuning_clear()
        sf.tuning_load(str(path))
        assert sf.tuning_size() == size
    finally:
        sf.tuning_clear()


def test_batched_workload_256():
    # the full uneven workload: 256 graphs, n log-uniform in [1e3, 5e4], one
    # launch, float sparse products, tol 1e-6; sampled graphs checked against
    # the oracle (implicit-nullspace ARPACK)
    sf = lib()
    specs = batched_specs()
    graphs = [batched_graph(s) for s in specs]
    ks = [s["k"] for s in specs]
    log(f"workload: {len(graphs)} graphs, sum n {sum(g.n for g in graphs)}, sum nnz {sum(g.nnz for g in graphs)}")
    Gs = [sf.Graph.from_msbm(g, False) for g in graphs]
    rs = sf.eigs_batched(Gs, ks, tol=1e-6, precision="mixed")
    paths = [r.info["path"] for r in rs]
    log(f"  launch ms {rs[0].info['batch_ms']:.2f}, graphs solved in the launch {paths.count(0)}")
    assert all(r.status in (sf.OK, sf.E_DEGENERATE) for r in rs), [r.status for r in rs]
    log(f"  degenerate (theta_k ~ theta_k+1): {sum(r.status == sf.E_DEGENERATE for r in rs)}")
    # every graph finished in the launch except the last few, handed off
    # (batch_status 5) to the single-graph solver with a warm start
    off = [i for i, r in enumerate(rs) if r.info["path"] != 0]
    assert len(off) <= 3 and all(rs[i].info["batch_status"] == 5 for i in off), [(i, rs[i].info) for i in off]
    # every member against the oracle's residual and the fairness and
    # orthonormality constraints (not the library's own residual figure)
    worst = 0.0
    for i, (g, k, r) in enumerate(zip(graphs, ks, rs)):
        W = g.to_scipy()
        H = to_np(r.H)
        lam = r.eigenvalues
        sigma = Gs[i].sigma
        assert np.all(np.diff(lam) >= -1e-12 * sigma), i
        F = oracle.fairness_matrix(g.groups, g.h)
        assert np.abs(F.T @ H).max() <= 1e-10 * np.sqrt(g.n) * np.abs(H).max(), i
        assert np.abs(H.T @ H - np.eye(k)).max() <= 1e-9, i
        res = oracle.residual_norms(W, g.groups, g.h, False, lam, H)
        worst = max(worst, res.max() / sigma)
        assert res.max() <= 1e-6 * sigma + 2e-12 * sigma, (i, res.max() / sigma)
    log(f"  all 256: worst oracle residual / sigma {worst:.2e}")
    # eigenvalues against the implicit-nullspace oracle on a sample (the
    # smallest and largest graphs, four at random and the handed-off ones)
    handed = set(off)
    order = np.argsort([g.n for g in graphs])
    rng = np.random.default_rng(3)
    sample = sorted(set([int(order[0]), int(order[-1])] + [int(x) for x in rng.choice(len(graphs), 4, replace=False)])
                    | handed)
    for i in sample:
        g, k, r = graphs[i], ks[i], rs[i]
        lam_ref, _ = oracle.fair_eigs_implicit(g.to_scipy(), g.groups, g.h, k, False, tol=1e-12)
        err = eig_parity(r.eigenvalues, lam_ref, 1e-5)
        log(f"  graph {i}: n={g.n} k={k} h={g.h} eig rel err {err:.2e}")
        assert err <= 1e-5
