"""Clustering metrics and subspace comparison (oracle side; test infrastructure).

* Error rate (Section 4.1, eq. err): the fraction of misclustered vertices
  under the best matching of computed to planted clusters.  Written with
  cluster indicator matrices the paper's expression counts every misclustered
  vertex twice (one wrong 1 and one missing 1 in the Frobenius norm), so the
  fraction is half of it; `error_rate(..., paper_scale=True)` returns the
  literal expression.
* Balance and average balance (Section 4.2, eq. bal / eq. avebal); a cluster
  missing some group has balance 0.
* Largest principal angle between two column spans, optionally in the
  D-weighted inner product of the normalized variant.
"""

from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linear_sum_assignment

__all__ = [
    "confusion",
    "error_rate",
    "error_rate_bruteforce",
    "balance",
    "average_balance",
    "max_principal_angle",
    "same_partition",
]


def confusion(pred, truth, k=None):
    pred = np.asarray(pred)
    truth = np.asarray(truth)
    if k is None:
        k = int(max(pred.max(), truth.max())) + 1
    M = np.zeros((k, k), dtype=np.int64)
    np.add.at(M, (pred, truth), 1)
    return M


def error_rate(pred, truth, k=None, paper_scale=False):
    """min over permutations of the misclustered fraction (Hungarian)."""
    M = confusion(pred, truth, k)
    r, c = linear_sum_assignment(-M)
    frac = 1.0 - M[r, c].sum() / len(pred)
    return 2.0 * frac if paper_scale else frac


def error_rate_bruteforce(pred, truth, k, paper_scale=False):
    """Same as error_rate by enumerating all k! permutation matrices J and
    evaluating ||H_hat J - H||_F^2 / n literally (small k only)."""
    pred = np.asarray(pred)
    truth = np.asarray(truth)
    n = len(pred)
    Hh = np.zeros((n, k))
    Hh[np.arange(n), pred] = 1
    H = np.zeros((n, k))
    H[np.arange(n), truth] = 1
    best = np.inf
    for perm in itertools.permutations(range(k)):
        J = np.zeros((k, k))
        J[np.arange(k), list(perm)] = 1
        best = min(best, np.sum((Hh @ J - H) ** 2) / n)
    return best if paper_scale else best / 2.0


def balance(labels, groups, h, k):
    """Balance(C_l) = min over s != s' of |V_s cap C_l| / |V_s' cap C_l|."""
    labels = np.asarray(labels)
    groups = np.asarray(groups)
    out = np.zeros(k)
    for l in range(k):
        cnt = np.bincount(groups[labels == l], minlength=h).astype(np.float64)
        if cnt.min() == 0:
            out[l] = 0.0
            continue
        best = np.inf
        for s in range(h):
            for s2 in range(h):
                if s != s2:
                    best = min(best, cnt[s] / cnt[s2])
        out[l] = best
    return out


def average_balance(labels, groups, h, k):
    return float(balance(labels, groups, h, k).mean())


def max_principal_angle(A, B, weights=None):
    """Largest principal angle between span(A) and span(B) (radians).

    With `weights` = d the angle is measured in the inner product <x, y>_D;
    computed as arcsin of ||Q_B - Q_A Q_A^T Q_B||_2 for accuracy at small
    angles.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if weights is not None:
        s = np.sqrt(np.asarray(weights, dtype=np.float64))[:, None]
        A = A * s
        B = B * s
    Qa, _ = np.linalg.qr(A)
    Qb, _ = np.linalg.qr(B)
    R = Qb - Qa @ (Qa.T @ Qb)
    s = np.linalg.norm(R, 2)
    return float(np.arcsin(min(1.0, s)))


def same_partition(a, b):
    """True iff labels a and b define the same partition (equal up to renaming)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.shape != b.shape:
        return False
    fwd = {}
    bwd = {}
    for x, y in zip(a.tolist(), b.tolist()):
        if fwd.setdefault(x, y) != y or bwd.setdefault(y, x) != x:
            return False
    return True
