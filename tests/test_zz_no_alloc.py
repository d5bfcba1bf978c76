"""The no-allocation operator entry point against the allocating one (GPU).

sfairsc_apply_operator_noalloc applies the same deflated operator
L^sigma = P (L_n - sigma I) P + sigma I (eq. asigma, Section 3.4 matvec)
through the same kernels and launch shapes as sfairsc_apply_operator, with
its scratch in a fixed device array.  Its output must equal the allocating
entry point's bit for bit, and the oracle's within the operator tolerance
(derivation in test_gpu_operator.py).  Consecutive calls with different
graphs and widths check that nothing carries over in the shared scratch;
sizes beyond the array and general constraints are refused without a launch.
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_common import lib, log, to_np
from sfairsc_inputs import random_sparse_graph, workload

pytestmark = pytest.mark.gpu


def _mixed_tol(g):
    deg_max = int(np.diff(g.rowptr).max())
    return 2.0 * (deg_max + 2) * 2.0**-24


def _check(sf, g, normalized, b, precision, seed):
    G = sf.Graph.from_msbm(g, normalized)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((g.n, b))
    Xd = torch.from_numpy(X).to("cuda")
    Y_ref = G.apply_operator(Xd, precision)
    # fill the output with garbage: the entry point must overwrite all of it
    Y = torch.full_like(Xd, float("nan"))
    G.apply_operator_noalloc(Xd, Y, precision)
    torch.cuda.synchronize()
    Yn, Yr = to_np(Y), to_np(Y_ref)
    assert np.array_equal(Yn, Yr), np.abs(Yn - Yr).max()
    ref = oracle.apply_deflated_operator(g.to_scipy(), g.groups, g.h, normalized, G.sigma, X)
    tol = 1e-12 if precision == "fp64" else _mixed_tol(g)
    assert np.abs(Yn - ref).max() <= tol * G.sigma * np.abs(X).max()
    return G


def test_noalloc_matches_the_allocating_entry_point():
    sf = lib()
    log("noalloc: msbm-2k-h2 normalized b=16 fp64, then er-1031-h3 b=3 mixed, then msbm-2k b=8 mixed")
    big = workload("msbm-2k-h2")
    small = random_sparse_graph(1031, 17, seed=1, h=3)
    _check(sf, big, True, 16, "fp64", 1)
    # second call: a smaller graph and a narrower (padded) block
    _check(sf, small, False, 3, "mixed", 2)
    # and back to the first graph with another width and precision
    _check(sf, big, True, 8, "mixed", 3)


def test_noalloc_refuses_what_does_not_fit():
    sf = lib()
    log("noalloc: refusals (scratch size, general constraint)")
    # 2 n BW 8 bytes of double blocks alone exceed 64 MiB at n = 140,000, b = 32
    g = random_sparse_graph(140_000, 4, seed=7, h=2)
    G = sf.Graph.from_msbm(g, False)
    X = torch.zeros((g.n, 32), dtype=torch.float64, device="cuda")
    Y = torch.full_like(X, 7.0)
    with pytest.raises(sf.SfairscError) as e:
        G.apply_operator_noalloc(X, Y, "fp64")
    assert e.value.code == sf._lib.E_ARG
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())
    # the same graph at b = 4 fits and agrees with the allocating entry point
    X4 = torch.from_numpy(np.random.default_rng(4).standard_normal((g.n, 4))).to("cuda")
    Y4 = torch.empty_like(X4)
    G.apply_operator_noalloc(X4, Y4, "fp64")
    assert torch.equal(Y4, G.apply_operator(X4, "fp64"))
    # a general constraint is not served without allocation
    small = random_sparse_graph(300, 8, seed=3, h=2)
    Gs = sf.Graph.from_msbm(small, False)
    Gs.set_constraint(np.random.default_rng(5).random((small.n, 2)))
    Xs = torch.zeros((small.n, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(sf.SfairscError) as e:
        Gs.apply_operator_noalloc(Xs, torch.empty_like(Xs), "fp64")
    assert e.value.code == sf._lib.E_ARG
