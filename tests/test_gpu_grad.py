"""The eigenvalue-sum gradient kernel (sfairsc_eigsum_backward) (GPU),
both variants.

Checked against (a) the oracle's analytic per-edge formula evaluated on the
oracle's own eigenvectors, (b) central finite differences of the GPU
forward (FP64), and (c) torch autograd through the FairEigSum function.
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


# --- normalized variant --------------------------------------------------------


def test_normalized_gradient_matches_oracle_formula_and_dense_reference():
    sf = lib()
    g = workload("msbm-500-h4-grad")
    k = 10
    lam, H = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, k + 1, True)
    assert lam[k] - lam[k - 1] > 1e-2
    G = sf.Graph.from_msbm(g, True)
    r = G.eigs(k, tol=1e-12, precision="fp64")
    assert np.allclose(r.eigenvalues, lam[:k], rtol=1e-10, atol=1e-12)
    grad = to_np(G.eigsum_backward(r.H, r.eigenvalues)).astype(np.float64)
    ref = oracle.eigsum_edge_gradient_normalized(g.rowptr, g.col, H[:, :k], lam[:k])
    rel = np.abs(grad - ref).max() / np.abs(ref).max()
    log(f"normalized gradient rel err {rel:.2e}")
    # FP32 output storage; the value depends only on the eigenspace
    assert rel <= 1e-6
    # on the kernel's own eigenvectors the formula holds to FP64 rounding
    # (FP64 values, FP64 output)
    G64 = sf.Graph(g.rowptr, g.col, torch.from_numpy(g.val.astype(np.float64)), g.groups, g.h, True)
    r64 = G64.eigs(k, tol=1e-12, precision="fp64")
    g64 = to_np(G64.eigsum_backward(r64.H, r64.eigenvalues))
    own = oracle.eigsum_edge_gradient_normalized(g.rowptr, g.col, to_np(r64.H), r64.eigenvalues)
    rel64 = np.abs(g64 - own).max() / np.abs(own).max()
    log(f"normalized gradient vs formula on the kernel's H: {rel64:.2e}")
    assert rel64 <= 1e-13


def test_normalized_gradient_central_differences():
    sf = lib()
    g = workload("msbm-500-h4-grad")
    k = 10
    vals = torch.from_numpy(g.val.astype(np.float64))
    rows = g.row_index()

    def f(v):
        G = sf.Graph(g.rowptr, g.col, v, g.groups, g.h, True)
        r = G.eigs(k, tol=1e-13, precision="fp64", max_restarts=4000)
        return float(np.sum(r.eigenvalues))

    G = sf.Graph(g.rowptr, g.col, vals, g.groups, g.h, True)
    r = G.eigs(k, tol=1e-13, precision="fp64")
    grad = to_np(G.eigsum_backward(r.H, r.eigenvalues))
    rng = np.random.default_rng(1)
    top = np.argsort(-np.abs(grad))[:3]
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
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-7


def test_normalized_fair_eigsum_autograd():
    sf = lib()
    g = workload("msbm-500-h4-grad")
    vals = torch.tensor(g.val, dtype=torch.float64, device="cuda", requires_grad=True)
    f = sf.FairEigSum.apply(vals, torch.from_numpy(g.rowptr), torch.from_numpy(g.col), torch.from_numpy(g.groups),
                            g.h, 5, 1e-12, True)
    f.backward()
    lam, H = oracle.fair_eigs_dense(g.to_scipy(), g.groups, g.h, 6, True)
    assert lam[5] - lam[4] > 1e-3
    assert float(f.detach()) == pytest.approx(lam[:5].sum(), rel=1e-10, abs=1e-12)
    ref = oracle.eigsum_edge_gradient_normalized(g.rowptr, g.col, H[:, :5], lam[:5])
    assert np.abs(to_np(vals.grad) - ref).max() <= 1e-8 * np.abs(ref).max()


def test_normalized_gradient_needs_eigenvalues():
    sf = lib()
    g = workload("msbm-500-h4-grad")
    G = sf.Graph.from_msbm(g, True)
    r = G.eigs(3, tol=1e-8, precision="fp64")
    with pytest.raises(sf.SfairscError) as e:
        G.eigsum_backward(r.H)
    assert e.value.code == sf.E_ARG
    with pytest.raises(ValueError):
        G.eigsum_backward(r.H, r.eigenvalues[:2])
