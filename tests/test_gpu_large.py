"""Full-size parity of the large workloads (GPU).

* n = 2,000,000 unnormalized modified SBM (k = 20, h = 8, average degree 30,
  weights U(0.5, 1.5)), float sparse products, tol 1e-6, block width 32.
  At this size the oracle's dense forms are out of reach, so the checks are
  the properties that fix the answer at any size: the oracle's own residual
  of every returned pair (||L^sigma x - theta x|| <= tol sigma, which with
  F^T H = 0 is the residual of the fair problem), F^T H = 0, H^T H = I,
  ascending eigenvalues in [0, sigma), and agreement with an FP64 solve of
  the same graph to the mixed bar (relative 1e-5).
* n = 200,000 gradient workload (k = 10, h = 4, degree 40): the backward
  kernel against the oracle's per-edge formula on every stored entry, and
  against central finite differences of the FP64 forward on 64 edges (32 of
  largest gradient, 32 at random).  The step is 1e-4: each eigenvalue of the
  shifted operator carries a rounding error of about eps * sigma, so the
  difference quotient's error is about k eps sigma / step; at this size the
  per-edge gradients are ~1e-5, and a 1e-6 step would leave an error of
  several percent, while 1e-4 leaves ~1e-3 relative (the n = 500 instance
  uses 1e-6, see test_gpu_grad).
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_common import eig_parity, lib, log, to_np
from sfairsc_inputs import workload

pytestmark = pytest.mark.gpu


def _fair_checks(g, lam, H, sigma, tol):
    W = g.to_scipy()
    F = oracle.fairness_matrix(g.groups, g.h)
    k = H.shape[1]
    assert np.all(np.diff(lam) >= -1e-12 * sigma)
    assert lam[0] >= -1e-9 * sigma and lam[-1] < sigma
    assert np.abs(F.T @ H).max() <= 1e-10 * np.sqrt(g.n) * np.abs(H).max()
    assert np.abs(H.T @ H - np.eye(k)).max() <= 1e-9
    res = oracle.residual_norms(W, g.groups, g.h, False, lam, H)
    log(f"  max residual / sigma {res.max() / sigma:.2e}")
    # the library's FP64 residual of a vector in null(C^T) is the oracle's
    assert res.max() <= tol * sigma + 2e-12 * sigma


def test_msbm_2m_mixed_full_size():
    sf = lib()
    g = workload("msbm-2m-h8")
    k, tol = 20, 1e-6
    log(f"msbm-2m: n={g.n} nnz={g.nnz}")
    G = sf.Graph.from_msbm(g, False)
    sigma = G.sigma
    r = G.eigs(k, tol=tol, precision="mixed", block_width=32)
    log(f"  mixed info {r.info}")
    lam, H = r.eigenvalues, to_np(r.H)
    _fair_checks(g, lam, H, sigma, tol)
    r64 = G.eigs(k, tol=1e-8, precision="fp64", block_width=32)
    err = eig_parity(lam, r64.eigenvalues, 1e-5)
    log(f"  mixed vs fp64 eigenvalue rel err {err:.2e}")
    assert err <= 1e-5


def test_gradient_200k_full_size():
    sf = lib()
    g = workload("msbm-200k-h4-grad")
    k = 10
    log(f"msbm-200k-grad: n={g.n} nnz={g.nnz}")
    vals = torch.from_numpy(g.val.astype(np.float64))
    G = sf.Graph(g.rowptr, g.col, vals, g.groups, g.h, False)
    sigma = G.sigma
    r = G.eigs(k, tol=1e-12, precision="fp64")
    log(f"  forward info {r.info}")
    H = to_np(r.H)
    grad = to_np(G.eigsum_backward(r.H))
    ref = oracle.eigsum_edge_gradient(g.rowptr, g.col, H)
    rel = np.abs(grad - ref).max() / np.abs(ref).max()
    log(f"  backward vs oracle formula rel err {rel:.2e}")
    assert rel <= 1e-12
    # warm start of the perturbed solves: the current eigenvectors
    x0 = r.H.contiguous()
    rows = g.row_index()

    def f(v):
        Gp = sf.Graph(g.rowptr, g.col, v, g.groups, g.h, False)
        # 1e-10: eigenvalue errors ~ (tol sigma)^2 / gap stay far below the
        # difference quotient's rounding term
        rp = Gp.eigs(k, tol=1e-10, precision="fp64", x0=x0)
        return float(np.sum(rp.eigenvalues))

    rng = np.random.default_rng(5)
    top = np.argsort(-grad)[:32]
    picks = list(top) + [int(x) for x in rng.choice(g.nnz, 32, replace=False)]
    step = 1e-4
    worst = 0.0
    for e in picks:
        i, j = rows[e], g.col[e]
        mate = g.rowptr[j] + np.searchsorted(g.col[g.rowptr[j]:g.rowptr[j + 1]], i)
        vp = vals.clone()
        vm = vals.clone()
        vp[e] += step
        vp[mate] += step
        vm[e] -= step
        vm[mate] -= step
        fd = (f(vp) - f(vm)) / (2 * step)
        an = grad[e] + grad[mate]
        bound = 1e-3 * abs(an) + 4 * k * 2.2e-16 * sigma / step
        worst = max(worst, abs(fd - an) / bound)
        assert abs(fd - an) <= bound, (e, fd, an)
    log(f"  finite differences: worst |fd - grad| / bound {worst:.2f}")


def test_normalized_gradient_200k_full_size():
    sf = lib()
    g = workload("msbm-200k-h4-grad")
    k = 10
    log(f"msbm-200k-grad normalized: n={g.n} nnz={g.nnz}")
    vals = torch.from_numpy(g.val.astype(np.float64))
    G = sf.Graph(g.rowptr, g.col, vals, g.groups, g.h, True)
    sigma = G.sigma
    r = G.eigs(k, tol=1e-12, precision="fp64")
    log(f"  forward info {r.info}")
    H, lam = to_np(r.H), r.eigenvalues
    grad = to_np(G.eigsum_backward(r.H, lam))
    ref = oracle.eigsum_edge_gradient_normalized(g.rowptr, g.col, H, lam)
    rel = np.abs(grad - ref).max() / np.abs(ref).max()
    log(f"  backward vs oracle formula rel err {rel:.2e}")
    assert rel <= 1e-12
    x0 = r.H.contiguous()
    rows = g.row_index()

    def f(v):
        Gp = sf.Graph(g.rowptr, g.col, v, g.groups, g.h, True)
        rp = Gp.eigs(k, tol=1e-10, precision="fp64", x0=x0)
        return float(np.sum(rp.eigenvalues))

    rng = np.random.default_rng(6)
    top = np.argsort(-np.abs(grad))[:8]
    picks = list(top) + [int(x) for x in rng.choice(g.nnz, 8, replace=False)]
    step = 1e-4
    worst = 0.0
    for e in picks:
        i, j = rows[e], g.col[e]
        mate = g.rowptr[j] + np.searchsorted(g.col[g.rowptr[j]:g.rowptr[j + 1]], i)
        vp = vals.clone()
        vm = vals.clone()
        vp[e] += step
        vp[mate] += step
        vm[e] -= step
        vm[mate] -= step
        fd = (f(vp) - f(vm)) / (2 * step)
        an = grad[e] + grad[mate]
        bound = 1e-3 * abs(an) + 4 * k * 2.2e-16 * sigma / step + 1e-10
        worst = max(worst, abs(fd - an) / bound)
        assert abs(fd - an) <= bound, (e, fd, an)
    log(f"  finite differences: worst |fd - grad| / bound {worst:.2f}")
