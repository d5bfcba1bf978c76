"""Pins of the oracle's Rayleigh-Ritz eigensolve (CPU only): closed-form
spectra of the shapes the projected matrix takes."""

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("n", [1, 2, 7, 64, 192])
def test_tridiagonal_toeplitz_closed_form(n):
    # tridiag(b, a, b): eigenvalues a + 2 b cos(j pi / (n + 1)), eigenvector
    # entries sin(i j pi / (n + 1))
    a, b = 3.0, -1.25
    T = a * np.eye(n) + b * (np.eye(n, k=1) + np.eye(n, k=-1))
    w, Z = oracle.ritz_pairs(T, min(n, 5))
    j = np.arange(1, n + 1)
    lam = np.sort(a + 2 * b * np.cos(j * np.pi / (n + 1)))
    assert np.allclose(w, lam, atol=1e-13 * abs(a) * n)
    # the smallest (b < 0: j = 1) eigenvector is sin(i pi / (n + 1)), normalised
    v = np.sin(np.arange(1, n + 1) * np.pi / (n + 1))
    v /= np.linalg.norm(v)
    assert abs(abs(Z[:, 0] @ v) - 1.0) < 1e-12


def test_arrowhead_closed_form():
    # a thick restart leaves diag(theta) with a coupling row: [[D, u], [u^T, a]];
    # with u = e_j s its eigenvalues are those of D except theta_j, plus the
    # two of [[theta_j, s], [s, a]]
    theta = np.array([0.5, 1.0, 2.0, 4.0])
    s, a, j = 0.75, 3.0, 2
    T = np.zeros((5, 5))
    T[:4, :4] = np.diag(theta)
    T[j, 4] = T[4, j] = s
    T[4, 4] = a
    w, _ = oracle.ritz_pairs(T)
    tr, det = theta[j] + a, theta[j] * a - s * s
    pair = [(tr - np.sqrt(tr * tr - 4 * det)) / 2, (tr + np.sqrt(tr * tr - 4 * det)) / 2]
    assert np.allclose(w, np.sort(np.r_[np.delete(theta, j), pair]), atol=1e-14)


def test_permuted_diagonal_and_symmetrisation():
    rng = np.random.default_rng(0)
    d = rng.permutation(np.arange(10.0))
    w, Z = oracle.ritz_pairs(np.diag(d))
    assert np.array_equal(w, np.arange(10.0))
    assert np.allclose(np.abs(Z), np.eye(10)[np.argsort(d)].T)
    # only the symmetric part counts
    K = rng.standard_normal((10, 10))
    w2, _ = oracle.ritz_pairs(np.diag(d) + (K - K.T))
    assert np.allclose(w2, w, atol=1e-13)


def test_keep_rule():
    theta = np.arange(80.0)
    assert oracle.krylov_schur_keep(theta, 80, 10, 8, 80, 100.0) == (48, 48)
    # a cluster at the cut is kept whole
    th = theta.copy()
    th[43:52] = 45.0  # theta_44 = theta_45: the cut at 45 would split it
    assert oracle.krylov_schur_keep(th, 80, 10, 8, 80, 100.0)[0] == 52
    # never more than ncv - b
    assert oracle.krylov_schur_keep(theta, 80, 70, 8, 80, 100.0) == (72, 72)
