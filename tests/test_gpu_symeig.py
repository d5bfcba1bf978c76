"""Parity of the Rayleigh-Ritz kernel (the eigensolver's small dense symmetric
eigenproblem, run on the GPU at every restart) against the oracle's LAPACK
eigendecomposition (GPU).

Bars (both sides are backward stable in FP64): eigenvalues within
64 eps ||T|| c of the oracle's; eigenvectors with residual
||T z - w z|| <= 64 eps ||T|| sqrt(c) and Z^T Z = I to 1e-12; where the
eigenvalue is separated from its neighbours by a relative gap g, the vector
agrees with the oracle's to about eps / g (Davis-Kahan), checked for g >= 1e-6.
Shapes: random symmetric matrices of every order class (one, two and three
column slots per lane, ragged tails), the block-tridiagonal plus arrowhead
shape of the Krylov-Schur projected matrix, closed-form Toeplitz spectra,
clusters down to exact multiplicities, diagonal input (no reflector), and
extreme scales.
"""

import numpy as np
import pytest
import torch

import oracle
from gpu_common import lib, log

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _run(T, m=None):
    sf = lib()
    Td = torch.from_numpy(np.ascontiguousarray(T)).to("cuda")
    w, Z = sf.symeig(Td, m)
    return w.cpu().numpy(), Z.cpu().numpy()


def _check(T, m=None, gap_check=True):
    c = T.shape[0]
    m = c if m is None else m
    w, Z = _run(T, m)
    w_ref, Z_ref = oracle.ritz_pairs(T, m)
    S = 0.5 * (T + T.T)
    nrm = max(np.abs(np.linalg.eigvalsh(S)).max(), np.finfo(float).tiny)
    err = np.abs(w - w_ref).max() / nrm
    assert np.all(np.diff(w) >= -64 * EPS * nrm)
    assert err <= 64 * EPS * c, err
    if m:
        R = S @ Z - Z * w[None, :m]
        res = np.linalg.norm(R, axis=0).max() / nrm
        orth = np.abs(Z.T @ Z - np.eye(m)).max()
        assert res <= 64 * EPS * np.sqrt(c), res
        assert orth <= 1e-12, orth
        if gap_check:
            wall = np.r_[-np.inf, w_ref, np.inf]
            for j in range(m):
                g = min(wall[j + 1] - wall[j], wall[j + 2] - wall[j + 1]) / nrm
                if g >= 1e-6:
                    cosang = abs(Z[:, j] @ Z_ref[:, j])
                    assert 1 - cosang <= max(1e-12, 1e3 * (EPS / g) ** 2), (j, g, 1 - cosang)
    return err


@pytest.mark.parametrize("c", [1, 2, 3, 5, 16, 63, 64, 65, 80, 100, 127, 128, 129, 160, 191, 192])
def test_random_symmetric(c):
    rng = np.random.default_rng(c)
    A = rng.standard_normal((c, c))
    err = _check(A + A.T)
    log(f"  c={c} eigenvalue err / ||T|| {err:.2e}")


@pytest.mark.parametrize("c,m", [(80, 48), (192, 112), (64, 10), (129, 0)])
def test_partial_vectors(c, m):
    rng = np.random.default_rng(100 + c)
    A = rng.standard_normal((c, c))
    _check(A + A.T, m)


def _krylov_schur_shape(p, b, nblk, rng, scale=1.0):
    # diag(theta) (kept Ritz values), a b-row coupling block, then block
    # tridiagonal Lanczos blocks of width b
    c = p + b * nblk
    T = np.zeros((c, c))
    T[:p, :p] = np.diag(np.sort(rng.uniform(0, 1, p)) * scale)
    for blk in range(nblk):
        r0 = p + b * blk
        D = rng.standard_normal((b, b)) * scale
        T[r0:r0 + b, r0:r0 + b] = D + D.T
        if blk == 0:
            C = rng.standard_normal((b, p)) * 1e-3 * scale
            T[r0:r0 + b, :p] = C
            T[:p, r0:r0 + b] = C.T
        else:
            R = np.triu(rng.standard_normal((b, b))) * scale
            T[r0:r0 + b, r0 - b:r0] = R
            T[r0 - b:r0, r0:r0 + b] = R.T
    return T


@pytest.mark.parametrize("p,b,nblk", [(48, 8, 4), (20, 4, 10), (96, 32, 3), (0, 8, 10), (160, 32, 1)])
def test_krylov_schur_shape(p, b, nblk):
    rng = np.random.default_rng(p + 7 * b + nblk)
    _check(_krylov_schur_shape(p, b, nblk, rng))


@pytest.mark.parametrize("c", [2, 50, 192])
def test_toeplitz_closed_form(c):
    a, b = 2.0, -1.0
    T = a * np.eye(c) + b * (np.eye(c, k=1) + np.eye(c, k=-1))
    w, Z = _run(T)
    lam = np.sort(a + 2 * b * np.cos(np.arange(1, c + 1) * np.pi / (c + 1)))
    assert np.abs(w - lam).max() <= 64 * EPS * 4 * c


@pytest.mark.parametrize("gap", [0.0, 1e-14, 1e-10, 1e-6])
def test_clusters(gap):
    # eigenvalue clusters of size 6 with spacing `gap` (0: exact multiplicity)
    rng = np.random.default_rng(5)
    c = 120
    base = np.repeat(np.linspace(0.1, 1.0, 20), 6)
    lam = base + gap * np.tile(np.arange(6), 20)
    Q, _ = np.linalg.qr(rng.standard_normal((c, c)))
    T = (Q * lam) @ Q.T
    _check(T, gap_check=False)
    # each cluster's eigenspace matches the oracle's (largest principal angle)
    w, Z = _run(T)
    _, Zr = oracle.ritz_pairs(T)
    for cl in range(20):
        sl = slice(6 * cl, 6 * cl + 6)
        s = np.linalg.svd(Zr[:, sl].T @ Z[:, sl], compute_uv=False)
        assert s.min() >= 1 - 1e-9, (cl, 1 - s.min())


def test_diagonal_and_block_diagonal():
    rng = np.random.default_rng(9)
    _check(np.diag(rng.permutation(np.arange(70.0))), gap_check=False)
    B = np.zeros((96, 96))
    for s in range(0, 96, 12):
        A = rng.standard_normal((12, 12))
        B[s:s + 12, s:s + 12] = A + A.T
    _check(B)


@pytest.mark.parametrize("scale", [1e-150, 1e-8, 1e6, 1e150])
def test_scales(scale):
    rng = np.random.default_rng(11)
    A = rng.standard_normal((90, 90))
    _check((A + A.T) * scale)


def test_repeatable_and_arguments():
    sf = lib()
    rng = np.random.default_rng(3)
    A = rng.standard_normal((100, 100))
    T = torch.from_numpy(A + A.T).cuda()
    w1, Z1 = sf.symeig(T, 30)
    w2, Z2 = sf.symeig(T, 30)
    assert torch.equal(w1, w2) and torch.equal(Z1, Z2)
    for bad in (0, 193):
        with pytest.raises(sf.SfairscError) as e:
            sf.symeig(torch.zeros((bad, bad), dtype=torch.float64, device="cuda"))
        assert e.value.code == sf.E_ARG
