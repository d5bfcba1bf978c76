"""Device memory is returned (GPU): repeated cycles of graph creation, solves
in both precisions, k-means, the backward, a batched launch, general and
membership constraints, failed creations (validation errors), failed and
unconverged solves, and handle destruction leave the device's free memory
where the first cycle left it."""

import gc

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from gpu_common import lib, log
from sfairsc_inputs import random_sparse_graph
from sfairsc_inputs.general import overlapping_memberships

pytestmark = pytest.mark.gpu


def _free_bytes():
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return torch.cuda.mem_get_info()[0]


def _cycle(sf, g, F, M):
    G = sf.Graph.from_msbm(g, False)
    r = G.eigs(4, tol=1e-8)
    G.eigs(4, tol=1e-6, precision="mixed")
    G.labels(r.H, 4, n_restarts=2)
    G.eigsum_backward(r.H)
    G.apply_operator(torch.ones(g.n, 8, dtype=torch.float64, device="cuda"))
    # failures on a live handle
    with pytest.raises(sf.SfairscError):
        G.eigs(4, block_width=5)
    with pytest.raises(sf.SfairscError):
        G.eigs(g.n, tol=1e-8)
    G.eigs(4, tol=1e-15, max_restarts=1, raise_not_converged=False)
    G2 = sf.Graph.from_msbm(g, True)
    sf.eigs_batched([G, G2], [3, 4], tol=1e-8, precision="fp64")
    G2.set_constraint(torch.from_numpy(F))
    G2.eigs(3, tol=1e-8)
    G2.set_memberships(sp.csr_matrix(M), inner_tol=1e-12)
    G2.eigs(3, tol=1e-8)
    G.close()
    G2.close()
    # failed creations: an asymmetric weight, a label outside [0, h)
    bad = g.val.copy()
    bad[5] += 0.25
    with pytest.raises(sf.SfairscError):
        sf.Graph(g.rowptr, g.col, bad, g.groups, g.h, False)
    lab = g.groups.copy()
    lab[0] = g.h
    with pytest.raises(sf.SfairscError):
        sf.Graph(g.rowptr, g.col, g.val, lab, g.h, False)


def test_no_device_memory_leak_over_failures_and_destruction():
    sf = lib()
    g = random_sparse_graph(12000, 10, seed=5, h=3)
    F = np.random.default_rng(7).random((g.n, 4))
    M = overlapping_memberships(g.n, 5, 0.2, seed=3)
    # the first cycle sets up what lives as long as the process (runtime and
    # code objects, the library's per-device state); then three more
    _cycle(sf, g, F, M)
    base = _free_bytes()
    for it in range(3):
        _cycle(sf, g, F, M)
        now = _free_bytes()
        log(f"  cycle {it}: free memory {(now - base) / 2**20:+.1f} MiB against the first cycle")
    # the basis alone is 12000 x 76 doubles (7 MiB) and the operator's two
    # block buffers 3 MiB each: any of them left behind by three cycles
    # exceeds this
    assert base - now <= 4 << 20
