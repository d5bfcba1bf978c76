"""The eigenvalue-sum gradient kernel (sfairsc_eigsum_backward) (GPU).

Checked against (a) the oracle's analytic per-edge formula evaluated on the
oracle's own eigenvectors, (b) central finite differences of the GPU
forward (FP64, tolerance 1e-12), and (c) torch autograd through the
FairEigSum function.
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_common import lib, log, to_np
from sfairsc_inputs import workload

pytestmark = pytest.mark.gpu


def test_gradient_matches_oracle_formula_and_dense_reference():
    sf = lib()
    g = workload("msbm-500-h4-grad")
    k = 10
    lam, H = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, k + 1, False)
    assert lam[k] - lam[k - 1] > 1e-3
    G = sf.Graph.from_msbm(g, False)
    r = G.eigs(k, tol=1e-12)
    grad = to_np(G.eigsum_backward(r.H)).astype(np.float64)
    ref = oracle.eigsum_edge_gradient(g.rowptr, g.col, H[:, :k])
    # the per-edge value depends only on the eigenspace; FP32 output storage
    rel = np.abs(grad - ref).max() / np.abs(ref).max()
    log(f"gradient rel err {rel:.2e}")
    assert rel <= 1e-6


def test_gradient_central_differences():
    sf = lib()
    g = workload("msbm-500-h4-grad")
    k = 10
    vals = torch.from_numpy(g.val.astype(np.float64))
    rows = g.row_index()

    def f(v):
        G = sf.Graph(g.rowptr, g.col, v, g.groups, g.h, False)
        r = G.eigs(k, tol=1e-13, max_restarts=4000)
        return float(np.sum(r.eigenvalues))

    G = sf.Graph(g.rowptr, g.col, vals, g.groups, g.h, False)
    r = G.eigs(k, tol=1e-13)
    grad = to_np(G.eigsum_backward(r.H))
    rng = np.random.default_rng(0)
    top = np.argsort(-grad)[:3]
    picks = list(top) + list(rng.choice(g.nnz, 3, replace=False))
    step = 1e-6
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
        log(f"edge {e}: fd {fd:.9f} analytic {an:.9f}")
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-6


def test_fair_eigsum_autograd():
    sf = lib()
    g = workload("msbm-500-h4-grad")
    vals = torch.tensor(g.val, dtype=torch.float64, device="cuda", requires_grad=True)
    f = sf.FairEigSum.apply(vals, torch.from_numpy(g.rowptr), torch.from_numpy(g.col), torch.from_numpy(g.groups),
                            g.h, 5, 1e-12)
    f.backward()
    lam, H = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, 5, False)
    assert float(f.detach()) == pytest.approx(lam.sum(), rel=1e-10)
    ref = oracle.eigsum_edge_gradient(g.rowptr, g.col, H)
    assert np.abs(to_np(vals.grad) - ref).max() <= 1e-8 * np.abs(ref).max()
