"""Seeded inputs with a general constraint matrix (no method arithmetic).

* random_laplacian: the paper's random-Laplacian workload (Section 5,
  "Random Laplacian"): a random sparse symmetric weight matrix of density s
  and a uniform random n x m matrix that stands in for F (it carries no group
  information).
* overlapping_memberships: 0/1 group-membership indicators where a vertex may
  belong to several groups (the extension discussed in Section 6).
"""

from __future__ import annotations

import numpy as np

from .msbm import MSBMGraph, _csr_from_edges, _sample_block_pair


def random_laplacian(n: int, s: float, m: int, seed: int, val_dtype=np.float64):
    """(graph, F): W symmetric with zero diagonal, each unordered pair {i, j}
    an edge with probability s, weight uniform on (0, 1/2) (a uniform (0, 1)
    draw on the lower triangle, averaged with its transpose); F float64
    n x m, entries uniform on [0, 1).  A vertex left without an edge is
    joined to a uniformly drawn other vertex (weight from the same law), so
    D is positive definite.  graph.groups is all zero (h = 1)."""
    rng = np.random.Generator(np.random.Philox(int(seed)))
    ei, ej = _sample_block_pair(rng, 0, n, 0, n, True, float(s))
    deg = np.bincount(ei, minlength=n) + np.bincount(ej, minlength=n)
    lone = np.flatnonzero(deg == 0)
    if lone.size:
        other = (lone + rng.integers(1, n, size=lone.size)) % n
        lo = np.minimum(lone, other)
        hi = np.maximum(lone, other)
        codes = np.unique(np.concatenate([ei * n + ej, lo * n + hi]))
        ei, ej = codes // n, codes % n
    w = 0.5 * rng.random(ei.size)
    w[w == 0.0] = 0.25  # keep every drawn pair an edge
    rowptr, col, val = _csr_from_edges(n, ei, ej, w, val_dtype)
    g = MSBMGraph(
        n=n,
        rowptr=rowptr,
        col=col,
        val=val,
        groups=np.zeros(n, dtype=np.int32),
        clusters=np.zeros(n, dtype=np.int32),
        h=1,
        k=1,
        n_repaired=int(lone.size),
        meta={"workload": f"random-laplacian-n{n}-s{s}-m{m}", "seed": int(seed)},
    )
    F = rng.random((n, m))
    return g, F


def overlapping_memberships(n: int, h: int, overlap: float, seed: int, union_of=None) -> np.ndarray:
    """n x h float64 0/1 memberships: every vertex in one primary group
    (uniform), and with probability `overlap` also in a second, distinct one.
    Every group is non-empty.  union_of=(a, b) appends one more column equal
    to the union of groups a and b (so the memberships are linearly
    dependent whenever a and b share no vertex)."""
    rng = np.random.Generator(np.random.Philox(int(seed) + 91))
    G = np.zeros((n, h))
    prim = rng.integers(0, h, size=n)
    for s_ in range(h):
        prim[s_ % n] = s_ if not (prim == s_).any() else prim[s_ % n]
    G[np.arange(n), prim] = 1.0
    extra = rng.random(n) < overlap
    sec = (prim + rng.integers(1, h, size=n)) % h
    G[np.flatnonzero(extra), sec[extra]] = 1.0
    if union_of is not None:
        a, b = union_of
        G = np.concatenate([G, np.maximum(G[:, a], G[:, b])[:, None]], axis=1)
    return G
