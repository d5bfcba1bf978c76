"""The Rayleigh-Ritz step of the Krylov eigensolver, restated plainly (oracle;
test infrastructure only).

At every restart, the eigensolver behind Alg. 3 step 3 (MATLAB's eigs, an
ARPACK Krylov method) needs the eigenpairs of the small symmetric matrix the
Krylov basis projects the operator onto; the Ritz values are its eigenvalues
and the Ritz vectors follow from its eigenvectors.  The plain definition is a
dense symmetric eigendecomposition, done here by LAPACK (numpy.linalg.eigh)
as a single step, in FP64.  Pinned in tests/test_oracle_ritz.py against
closed-form spectra.
"""

from __future__ import annotations

import numpy as np

__all__ = ["ritz_pairs", "krylov_schur_keep"]


def ritz_pairs(T, m=None):
    """Eigenvalues (ascending) of the symmetric part of T and the unit
    eigenvectors of the m smallest (columns)."""
    T = np.asarray(T, dtype=np.float64)
    S = 0.5 * (T + T.T)
    w, Z = np.linalg.eigh(S)
    m = S.shape[0] if m is None else int(m)
    return w, Z[:, :m]


def krylov_schur_keep(theta, c, k, b, ncv, sigma, keep=0):
    """Number p of Ritz vectors a thick restart keeps (Krylov-Schur; the
    paper's ARPACK call restarts implicitly with a comparable count): at
    least k + b and half of the unwanted ones, at most ncv - b, extended while
    it would split a cluster of Ritz values equal to 1e-10 sigma, rounded up
    to a multiple of four; and m = max(p, k) Ritz vectors formed."""
    p = keep if keep > 0 else max(k + b, k + (c - k) // 2)
    p = min(p, ncv - b)
    p = max(p, min(k, ncv - b))
    while p < ncv - b and p < c and abs(theta[p] - theta[p - 1]) <= 1e-10 * sigma:
        p += 1
    p = min((p + 3) & ~3, ncv - b)
    return p, min(c, max(p, k))
