"""The float64 Jacobi eigensolver of the interpolation kernels against LAPACK
(numpy.linalg.eigvalsh) on matrices given directly: with the single lattice
vector R = 0 (degeneracy 1) the interpolated matrix at every k is H(R = 0)
itself.  Cases: random Hermitian matrices of every size 1..16 (odd sizes run
the padded round-robin schedule), clustered and exactly degenerate spectra,
couplings far below the rounding of the diagonal (down to 1e-200, where
|b|^2 is subnormal or zero), an exactly degenerate pair joined only by such a
coupling (a 45-degree rotation driven by a 1e-160 element), zero couplings,
and matrices scaled by 1e+-100.

Eigenvalues are compared with LAPACK; eigenvectors, not unique for
degenerate or clustered levels, are checked for what holds for any valid
choice: the residual H U - U diag(eps) and orthonormality.  Bounds, relative
to the Frobenius norm of H: eigenvalues 1e-13, residual 1e-12 (largest
entry), orthonormality 1e-13 (largest entry of U^H U - 1, absolute)."""
import sys

import numpy as np
import pytest
import torch

from paper_1604_03525_amd import epw

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _solve(H):
    R = np.zeros((1, 3), dtype=np.int32)
    nd = np.ones(1, dtype=np.int32)
    k = np.array([[0.1, 0.2, 0.3], [0.7, 0.0, 0.5]])
    eps, U = epw.epw_interp_bands(torch.as_tensor(H[None]).to(DEV), R, nd, k)
    eps, U = eps.cpu().numpy(), U.cpu().numpy()
    assert np.array_equal(eps[0], eps[1]) and np.array_equal(U[0], U[1])   # same matrix, same result
    return eps[0], U[0]


def _check(tag, H):
    n = H.shape[0]
    nrm = np.linalg.norm(H)
    eps, U = _solve(H)
    ref = np.linalg.eigvalsh(H)
    e_err = np.abs(eps - ref).max() / nrm
    res = np.abs(H @ U - U * eps).max() / nrm
    orth = np.abs(U.conj().T @ U - np.eye(n)).max()
    _say(tag, "n", n, "eig %.1e res %.1e orth %.1e" % (e_err, res, orth))
    assert np.all(np.diff(eps) >= 0)
    assert e_err < 1e-13 and res < 1e-12 and orth < 1e-13


def _random_hermitian(n, rng, scale=1.0):
    X = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return scale * (X + X.conj().T)


def _with_spectrum(ev, rng):
    n = len(ev)
    Q = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))[0]
    H = Q @ np.diag(ev) @ Q.conj().T
    return 0.5 * (H + H.conj().T)


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_random_every_size(n):
    rng = np.random.default_rng(100 + n)
    for rep in range(3):
        _check(("random", rep), _random_hermitian(n, rng))


@pytest.mark.parametrize("n", [7, 16])
def test_clustered_and_degenerate(n):
    rng = np.random.default_rng(200 + n)
    base = rng.uniform(-6.0, 6.0, n - 5)
    ev = np.sort(np.concatenate([base, [1.0, 1.0 + 1e-9, 1.0 + 2e-9, -2.0, -2.0]]))
    _check("clustered", _with_spectrum(ev, rng))
    _check("all equal", _with_spectrum(np.full(n, 0.75), rng))


@pytest.mark.parametrize("n", [6, 16])
def test_tiny_couplings(n):
    """A random 3 x 3 block keeps the sweeps going, so every pair is rotated,
    including those joined only by a tiny coupling: its phase must keep unit
    modulus or the rotated columns lose their norm."""
    rng = np.random.default_rng(300 + n)
    d = np.sort(rng.uniform(-3.0, 3.0, n))
    for mag in (1e-150, 1e-160, 1e-200, 0.0):
        H = np.diag(d).astype(np.complex128)
        H[:3, :3] = _random_hermitian(3, rng)
        for i in range(3, n - 1):
            H[i, i + 1] = mag * np.exp(2j * np.pi * rng.random())
            H[i + 1, i] = np.conj(H[i, i + 1])
        _check(("tiny coupling", mag), H)
    # an exactly degenerate pair joined only by a 1e-160 coupling: its rotation is
    # a full 45 degrees whose phase comes from the tiny element alone
    H = np.zeros((n, n), dtype=np.complex128)
    H[:3, :3] = _random_hermitian(3, rng)
    for i in range(3, n):
        H[i, i] = d[i]
    H[n - 1, n - 1] = H[n - 2, n - 2]
    H[n - 2, n - 1] = 1e-160 * np.exp(0.7j)
    H[n - 1, n - 2] = np.conj(H[n - 2, n - 1])
    _check("degenerate pair, tiny coupling", H)


@pytest.mark.parametrize("scale", [1e-100, 1e100])
def test_extreme_scales(scale):
    rng = np.random.default_rng(400)
    for n in (3, 16):
        _check(("scale", scale), _random_hermitian(n, rng, scale))
