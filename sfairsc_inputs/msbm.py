"""Modified stochastic block model (m-SBM) graphs, seeded and reproducible.

The m-SBM (paper, Appendix B.1, "m-SBM", eq. p-msbm / w-msbm) plants k clusters
and h groups.  Block (i, j) holds the u_i^(j) vertices that are in cluster i
and group j.  Vertices are numbered cluster-major, then group, as in the
paper's Example B.2, unless a relabelling is applied afterwards.  Every
unordered pair {v, w} with v != w is an edge independently with a probability
that depends only on whether v and w share a cluster and whether they share a
group; the graph is undirected and has no self-loops.

Probabilities are passed by *meaning* rather than by letter, because the two
sources disagree on which letter is which (the paper names the "different
cluster, same group" probability b and the "same cluster, different group"
probability c; the workload table below follows the opposite lettering):

    p_in_same   : same cluster, same group
    p_in_diff   : same cluster, different group
    p_out_same  : different cluster, same group
    p_out_diff  : different cluster, different group

Exact sampling.  For each unordered pair of blocks the number of edges is drawn
from Binomial(#pairs, p) and that many distinct pairs are then drawn uniformly
without replacement; this has exactly the distribution of independent
Bernoulli(p) trials per pair, at O(n + m) cost.  Randomness comes from numpy's
Philox counter-based generator keyed by the seed.

Isolated vertices (the paper assumes none) are repaired by joining each one to
a uniformly chosen vertex of its own block (its own cluster if the block is a
singleton); the number of repairs is recorded.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "MSBMGraph",
    "msbm",
    "msbm_from_blocks",
    "relabel",
    "workload",
    "WORKLOADS",
    "random_sparse_graph",
    "fair_block_sizes",
    "scale_for_degree",
]


@dataclasses.dataclass
class MSBMGraph:
    """An undirected weighted graph in CSR form plus its labels.

    rowptr int32[n+1], col int32[nnz] (sorted within each row), val float32 or
    float64 [nnz] holding both stored copies (i, j) and (j, i) of each edge.
    groups int32[n] in [0, h); clusters int32[n] in [0, k) (planted truth).
    """

    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    groups: np.ndarray
    clusters: np.ndarray
    h: int
    k: int
    n_repaired: int = 0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self, dtype=np.float64):
        import scipy.sparse as sp

        return sp.csr_matrix(
            (self.val.astype(dtype), self.col.astype(np.int64), self.rowptr.astype(np.int64)),
            shape=(self.n, self.n),
        )

    def row_index(self) -> np.ndarray:
        """Row index of every stored entry (int32[nnz])."""
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.rowptr))


# ----------------------------------------------------------------------------
# block-pair sampling


def _sample_distinct(rng: np.random.Generator, count: int, universe: int) -> np.ndarray:
    """`count` distinct integers drawn uniformly from [0, universe)."""
    if count <= 0:
        return np.zeros(0, dtype=np.int64)
    if count * 3 >= universe:
        # dense regime: a uniform random subset via a permutation prefix
        return rng.permutation(universe)[:count].astype(np.int64)
    got = np.unique(rng.integers(0, universe, size=count, dtype=np.int64))
    while got.size < count:
        extra = rng.integers(0, universe, size=2 * (count - got.size) + 16, dtype=np.int64)
        got = np.unique(np.concatenate([got, extra]))
    if got.size > count:
        got = rng.choice(got, size=count, replace=False)
    return np.sort(got)


def _sample_block_pair(rng, off1, s1, off2, s2, same_block, p):
    """Edges between two blocks (or inside one), as (i, j) arrays with i < j."""
    if p <= 0.0 or s1 == 0 or s2 == 0:
        z = np.zeros(0, dtype=np.int64)
        return z, z
    if same_block:
        npairs = s1 * (s1 - 1) // 2
        if npairs == 0:
            z = np.zeros(0, dtype=np.int64)
            return z, z
        m = int(rng.binomial(npairs, min(p, 1.0)))
        if npairs <= 5_000_000:
            iu, ju = np.triu_indices(s1, 1)
            pick = _sample_distinct(rng, m, npairs)
            return off1 + iu[pick].astype(np.int64), off1 + ju[pick].astype(np.int64)
        # large sparse block: ordered draws mapped to unordered pairs are
        # uniform over unordered pairs; dedupe and top up to exactly m.
        codes = np.zeros(0, dtype=np.int64)
        while codes.size < m:
            need = m - codes.size
            a = rng.integers(0, s1, size=2 * need + 16, dtype=np.int64)
            b = rng.integers(0, s1, size=2 * need + 16, dtype=np.int64)
            keep = a != b
            lo = np.minimum(a[keep], b[keep])
            hi = np.maximum(a[keep], b[keep])
            codes = np.unique(np.concatenate([codes, lo * s1 + hi]))
        if codes.size > m:
            codes = np.sort(rng.choice(codes, size=m, replace=False))
        return off1 + codes // s1, off1 + codes % s1
    npairs = s1 * s2
    m = int(rng.binomial(npairs, min(p, 1.0)))
    idx = _sample_distinct(rng, m, npairs)
    return off1 + idx // s2, off2 + idx % s2


def _csr_from_edges(n, ei, ej, w, val_dtype):
    rows = np.concatenate([ei, ej])
    cols = np.concatenate([ej, ei])
    vals = np.concatenate([w, w]).astype(val_dtype)
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    rows = rows[order]
    cols = cols[order]
    vals = vals[order]
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("graph too large for int32 CSR indices")
    return rowptr.astype(np.int32), cols.astype(np.int32), vals


def fair_block_sizes(cluster_sizes: Sequence[int], group_fracs: Sequence[float]) -> np.ndarray:
    """k x h block sizes u_i^(j): each cluster split by the group fractions.

    Uses largest-remainder rounding per cluster, so a cluster whose size times
    every fraction is an integer is split exactly (the fair layout of the
    paper's eq. fair-block).
    """
    fr = np.asarray(group_fracs, dtype=np.float64)
    fr = fr / fr.sum()
    out = np.zeros((len(cluster_sizes), len(fr)), dtype=np.int64)
    for i, cs in enumerate(cluster_sizes):
        raw = cs * fr
        base = np.floor(raw + 1e-9).astype(np.int64)
        rem = cs - base.sum()
        order = np.argsort(-(raw - base), kind="stable")
        base[order[:rem]] += 1
        out[i] = base
    return out


def _expected_avg_degree(u: np.ndarray, probs) -> float:
    k, h = u.shape
    p_in_same, p_in_diff, p_out_same, p_out_diff = probs
    n = u.sum()
    tot = 0.0
    for i in range(k):
        for j in range(h):
            s = u[i, j]
            if s == 0:
                continue
            deg = 0.0
            for i2 in range(k):
                for j2 in range(h):
                    s2 = u[i2, j2] - (1 if (i2 == i and j2 == j) else 0)
                    if i2 == i:
                        p = p_in_same if j2 == j else p_in_diff
                    else:
                        p = p_out_same if j2 == j else p_out_diff
                    deg += s2 * p
            tot += s * deg
    return tot / n


def scale_for_degree(u: np.ndarray, ratios, avg_degree: float) -> tuple:
    """Scale probability ratios so that the expected average degree matches."""
    base = _expected_avg_degree(np.asarray(u), tuple(ratios))
    s = avg_degree / base
    return tuple(float(r) * s for r in ratios)


def msbm_from_blocks(
    u,
    probs,
    seed: int,
    weights=("unit",),
    repair_isolated: bool = True,
    val_dtype=np.float64,
) -> MSBMGraph:
    """m-SBM graph from a k x h block-size matrix u (vertices in block order).

    probs = (p_in_same, p_in_diff, p_out_same, p_out_diff).
    weights: ("unit",) -> 1.0; ("alpha_beta", alpha, beta) -> alpha within a
    cluster and beta between clusters (the paper's eq. msbm-bernoulli);
    ("uniform", lo, hi) -> Uniform(lo, hi) drawn in float32 per edge.
    """
    u = np.asarray(u, dtype=np.int64)
    k, h = u.shape
    n = int(u.sum())
    rng = np.random.Generator(np.random.Philox(int(seed)))
    p_in_same, p_in_diff, p_out_same, p_out_diff = (float(x) for x in probs)

    offs = np.zeros(k * h + 1, dtype=np.int64)
    np.cumsum(u.reshape(-1), out=offs[1:])
    clusters = np.repeat(np.repeat(np.arange(k, dtype=np.int32), h), u.reshape(-1))
    groups = np.repeat(np.tile(np.arange(h, dtype=np.int32), k), u.reshape(-1))

    ei_parts, ej_parts, w_parts = [], [], []
    nb = k * h
    for b1 in range(nb):
        c1, g1 = divmod(b1, h)
        for b2 in range(b1, nb):
            c2, g2 = divmod(b2, h)
            if c1 == c2:
                p = p_in_same if g1 == g2 else p_in_diff
            else:
                p = p_out_same if g1 == g2 else p_out_diff
            ei, ej = _sample_block_pair(
                rng, offs[b1], u[c1, g1], offs[b2], u[c2, g2], b1 == b2, p
            )
            if ei.size == 0:
                continue
            ei_parts.append(ei)
            ej_parts.append(ej)
            within = c1 == c2
            if weights[0] == "unit":
                w = np.ones(ei.size, dtype=np.float64)
            elif weights[0] == "alpha_beta":
                w = np.full(ei.size, float(weights[1] if within else weights[2]))
            elif weights[0] == "uniform":
                w = None  # drawn after concatenation, in edge order
            else:
                raise ValueError(f"unknown weights {weights!r}")
            w_parts.append(w)

    ei = np.concatenate(ei_parts) if ei_parts else np.zeros(0, np.int64)
    ej = np.concatenate(ej_parts) if ej_parts else np.zeros(0, np.int64)
    if weights[0] == "uniform":
        lo, hi = float(weights[1]), float(weights[2])
        w = (lo + (hi - lo) * rng.random(ei.size, dtype=np.float32)).astype(np.float32)
        val_dtype = np.float32
    else:
        w = np.concatenate(w_parts) if w_parts else np.zeros(0)

    n_rep = 0
    if repair_isolated and n > 1:
        deg = np.bincount(ei, minlength=n) + np.bincount(ej, minlength=n)
        iso = np.flatnonzero(deg == 0)
        add_i, add_j = [], []
        for v in iso:
            b = int(np.searchsorted(offs, v, side="right") - 1)
            lo_b, hi_b = offs[b], offs[b + 1]
            if hi_b - lo_b >= 2:
                cand_lo, cand_hi = lo_b, hi_b
            else:
                c = b // h
                cand_lo, cand_hi = offs[c * h], offs[(c + 1) * h]
                if cand_hi - cand_lo < 2:
                    cand_lo, cand_hi = 0, n
            while True:
                t = int(rng.integers(cand_lo, cand_hi))
                if t != v:
                    break
            add_i.append(min(v, t))
            add_j.append(max(v, t))
        if add_i:
            # a partner may itself have been isolated and already joined: dedupe
            pairs = np.unique(np.stack([np.array(add_i), np.array(add_j)], 1), axis=0)
            n_rep = int(iso.size)
            ei = np.concatenate([ei, pairs[:, 0]])
            ej = np.concatenate([ej, pairs[:, 1]])
            w_add = np.ones(pairs.shape[0], dtype=w.dtype)
            if weights[0] == "alpha_beta":
                w_add[:] = float(weights[1])
            w = np.concatenate([w, w_add])

    rowptr, col, val = _csr_from_edges(n, ei, ej, w, val_dtype)
    return MSBMGraph(
        n=n,
        rowptr=rowptr,
        col=col,
        val=val,
        groups=groups,
        clusters=clusters,
        h=h,
        k=k,
        n_repaired=n_rep,
        meta={"u": u.tolist(), "probs": list(map(float, probs)), "weights": list(weights), "seed": int(seed)},
    )


def msbm(n, k, h, probs, seed, group_fracs=None, weights=("unit",), val_dtype=np.float64):
    """m-SBM with k equal clusters (sizes differ by at most one) split by group fractions."""
    base, extra = divmod(int(n), int(k))
    sizes = [base + (1 if i < extra else 0) for i in range(k)]
    fr = group_fracs if group_fracs is not None else [1.0] * h
    u = fair_block_sizes(sizes, fr)
    return msbm_from_blocks(u, probs, seed, weights=weights, val_dtype=val_dtype)


def relabel(g: MSBMGraph, seed: int) -> MSBMGraph:
    """Apply a seeded uniformly random vertex relabelling (new id = perm[old])."""
    rng = np.random.Generator(np.random.Philox(int(seed) ^ 0x5EED))
    perm = rng.permutation(g.n).astype(np.int64)
    rows = perm[g.row_index().astype(np.int64)]
    cols = perm[g.col.astype(np.int64)]
    key = rows * g.n + cols
    order = np.argsort(key, kind="stable")
    counts = np.bincount(rows, minlength=g.n)
    rowptr = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    groups = np.empty_like(g.groups)
    clusters = np.empty_like(g.clusters)
    groups[perm] = g.groups
    clusters[perm] = g.clusters
    meta = dict(g.meta)
    meta["relabel_seed"] = int(seed)
    return MSBMGraph(
        n=g.n,
        rowptr=rowptr.astype(np.int32),
        col=cols[order].astype(np.int32),
        val=g.val[order],
        groups=groups,
        clusters=clusters,
        h=g.h,
        k=g.k,
        n_repaired=g.n_repaired,
        meta=meta,
    )


def random_sparse_graph(n, avg_degree, seed, h=2, weights=("uniform", 0.5, 1.5), val_dtype=np.float64):
    """Erdos-Renyi graph G(n, p) with p = avg_degree/(n-1) and random group labels.

    Groups are drawn iid uniform in [0, h) and then forced non-empty.  This is
    a structure-free workload for operator and kernel tests.
    """
    p = min(1.0, float(avg_degree) / max(n - 1, 1))
    g = msbm_from_blocks(np.array([[n]]), (p, p, p, p), seed, weights=weights, val_dtype=val_dtype)
    rng = np.random.Generator(np.random.Philox(int(seed) + 7777))
    groups = rng.integers(0, h, size=n).astype(np.int32)
    for s in range(h):
        if not (groups == s).any():
            groups[s % n] = s
    g.groups = groups
    g.h = h
    g.k = 1
    return g


# ----------------------------------------------------------------------------
# named workloads (synthetic stand-ins for the paper's m-SBM experiments)


def _w_2k(seed=1):
    u = fair_block_sizes([400] * 5, [1, 1])
    return msbm_from_blocks(u, (0.20, 0.15, 0.05, 0.02), seed)


def _w_50k(seed=2):
    u = np.array([[2000, 1250, 750, 500, 500]] * 10)
    return msbm_from_blocks(u, (8e-3, 6e-3, 2e-3, 5e-4), seed)


def _w_2m(seed=3):
    u = fair_block_sizes([100000] * 20, [1] * 8)
    f = 30.0 / 14.912
    probs = (1.2e-4 * f, 8e-5 * f, 6e-6 * f, 3e-6 * f)
    return msbm_from_blocks(u, probs, seed, weights=("uniform", 0.5, 1.5))


def _w_200k(seed=5):
    u = fair_block_sizes([20000] * 10, [1] * 4)
    probs = scale_for_degree(u, (4.0, 3.0, 1.0, 0.5), 40.0)
    return msbm_from_blocks(u, probs, seed, weights=("uniform", 0.5, 1.5))


def _w_500(seed=55):
    u = fair_block_sizes([50] * 10, [1] * 4)
    probs = scale_for_degree(u, (4.0, 3.0, 1.0, 0.5), 40.0)
    return msbm_from_blocks(u, probs, seed, weights=("uniform", 0.5, 1.5))


# name -> (builder, solve parameters)
WORKLOADS = {
    "msbm-2k-h2": (_w_2k, dict(k=5, normalized=False, tol=1e-10, block=8)),
    "msbm-50k-h5-normalized": (_w_50k, dict(k=10, normalized=True, tol=1e-8, block=8)),
    "msbm-2m-h8": (_w_2m, dict(k=20, normalized=False, tol=1e-6, block=32)),
    "msbm-200k-h4-grad": (_w_200k, dict(k=10, normalized=False, tol=1e-10, block=8)),
    "msbm-500-h4-grad": (_w_500, dict(k=10, normalized=False, tol=1e-12, block=8)),
}


def workload(name: str, relabel_seed: Optional[int] = None) -> MSBMGraph:
    """Build a named workload; optionally apply a seeded random relabelling."""
    g = WORKLOADS[name][0]()
    g.meta["workload"] = name
    if relabel_seed is not None:
        g = relabel(g, relabel_seed)
    return g


def batched_specs(count=256, seed=4):
    """Per-graph parameters of the uneven batched workload.

    n log-uniform in [1000, 50000], k uniform in {2..10}, h uniform in {2..6}
    (equal groups), average degree uniform in [10, 80], probability ratios
    4 : 3 : 1 : 0.5 (same cluster same group : same cluster different group :
    different cluster same group : neither).
    """
    rng = np.random.Generator(np.random.Philox(int(seed)))
    specs = []
    for t in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1000), math.log(50000)))))
        k = int(rng.integers(2, 11))
        h = int(rng.integers(2, 7))
        deg = float(rng.uniform(10, 80))
        specs.append(dict(n=n, k=k, h=h, avg_degree=deg, seed=int(seed) * 100003 + t))
    return specs


def batched_graph(spec) -> MSBMGraph:
    n, k, h = spec["n"], spec["k"], spec["h"]
    base, extra = divmod(n, k)
    sizes = [base + (1 if i < extra else 0) for i in range(k)]
    u = fair_block_sizes(sizes, [1] * h)
    probs = scale_for_degree(u, (4.0, 3.0, 1.0, 0.5), spec["avg_degree"])
    return msbm_from_blocks(u, probs, spec["seed"])
