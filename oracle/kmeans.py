"""k-means on the rows of H (Alg. 3 step 4), oracle side (test infrastructure).

The paper says only "apply k-means clustering to the rows of H".  The reading
used here (and, independently, by the GPU library) is:

* input: the n rows of H as points in R^kdim, no row normalisation;
* seeding: k-means++ D^2 sampling (Arthur and Vassilvitskii, 2007).  Draw t of
  restart r is the SplitMix64 uniform u(seed, r, t).  The first centre is row
  floor(u * n).  Centre t >= 1 is the first row i whose inclusive prefix sum of
  D^2 (squared distance to the nearest chosen centre) exceeds u * total; if
  total is 0 the row floor(u * n) is taken;
* Lloyd: assign every row to its nearest centroid by squared Euclidean
  distance (ties: lowest centroid index); stop when no label changes or after
  max_iter assignments; otherwise move each centroid to the mean of its rows.
  A centroid left with no rows is moved to the row farthest from its own
  centroid (ties: lowest row index), processed in increasing cluster order,
  each chosen row being used at most once;
* restarts: keep the lowest inertia (sum of squared distances of the final
  assignment), ties to the lowest restart index; then renumber the labels in
  order of first appearance.

Lloyd's steps only use distances and means, which are unchanged by an
orthogonal change of basis of the columns of H; clustering therefore does not
depend on the sign or rotation freedom of the eigenvectors.
"""

from __future__ import annotations

import numpy as np

from .splitmix import splitmix64_uniform

__all__ = ["kmeans_pp_seeds", "lloyd", "kmeans", "first_appearance"]


def _sqdist(X, c):
    diff = X - c[None, :]
    return np.einsum("ij,ij->i", diff, diff)


def kmeans_pp_seeds(X, k, seed, restart):
    """Row indices of the k-means++ seeds for one restart."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    u = splitmix64_uniform(seed, restart, 0)
    idx = [min(int(u * n), n - 1)]
    d2 = _sqdist(X, X[idx[0]])
    for t in range(1, k):
        u = splitmix64_uniform(seed, restart, t)
        cs = np.cumsum(d2)
        total = cs[-1]
        if total > 0.0:
            i = int(np.searchsorted(cs, u * total, side="right"))
            i = min(i, n - 1)
        else:
            i = min(int(u * n), n - 1)
        idx.append(i)
        d2 = np.minimum(d2, _sqdist(X, X[i]))
    return idx


def lloyd(X, centroids, max_iter=300):
    """Lloyd iterations from given centroids -> (labels, inertia, n_assign)."""
    X = np.asarray(X, dtype=np.float64)
    C = np.array(centroids, dtype=np.float64, copy=True)
    n = X.shape[0]
    k = C.shape[0]
    labels = np.full(n, -1, dtype=np.int64)
    mind = None
    it = 0
    while it < max_iter:
        D = np.stack([_sqdist(X, C[j]) for j in range(k)], axis=1)
        new = np.argmin(D, axis=1)  # first minimum: lowest index on ties
        mind = D[np.arange(n), new]
        changed = int(np.count_nonzero(new != labels))
        labels = new
        it += 1
        if changed == 0 or it == max_iter:
            break
        for j in range(k):
            rows = labels == j
            if rows.any():
                C[j] = X[rows].mean(axis=0)
        used = np.zeros(n, dtype=bool)
        far = mind.copy()
        for j in range(k):
            if not np.any(labels == j):
                cand = np.where(used, -np.inf, far)
                i = int(np.argmax(cand))
                C[j] = X[i]
                used[i] = True
    return labels, float(mind.sum()), it


def first_appearance(labels):
    """Renumber labels in order of first appearance."""
    labels = np.asarray(labels)
    out = np.empty_like(labels)
    mapping = {}
    for i, l in enumerate(labels.tolist()):
        if l not in mapping:
            mapping[l] = len(mapping)
        out[i] = mapping[l]
    return out


def kmeans(X, k, n_restarts=10, seed=0, max_iter=300):
    """Best-of-restarts k-means -> (labels int32[n], inertia)."""
    X = np.asarray(X, dtype=np.float64)
    best = None
    for r in range(n_restarts):
        idx = kmeans_pp_seeds(X, k, seed, r)
        labels, inertia, _ = lloyd(X, X[idx], max_iter)
        if best is None or inertia < best[1]:
            best = (labels, inertia)
    return first_appearance(best[0]).astype(np.int32), best[1]
