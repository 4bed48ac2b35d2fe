"""Wannier-Fourier interpolation from real space onto fine k/q points
(oracle side, plain NumPy float64).

Test infrastructure only (see oracle/__init__.py).

The paper names this interpolation as the most time-consuming stage of the
code (Sec. 8, Fig. "Speedup" and the strong-scaling discussion) and takes
its equations from the cited Giustino 2007 work without printing them.  The
reading used here, written out so it can be checked by eye:

  X(p) = sum_R exp(+2 pi i p.R) X(R) / ndeg(R)          (p fractional, R integer)
  H(k) -> Hermitised (H + H^dagger)/2 -> eigh -> eps_nk ascending, U_k columns
  D(q) -> Hermitised -> eigh -> lambda_nu, omega_nu = sign(lambda) sqrt|lambda|,
          e_q columns (masses already folded into D: Sec. 3, below Eq. (2))
  g_ka(k,q) = sum_{R_e} sum_{R_p} exp(2 pi i (k.R_e + q.R_p)) g_ka(R_e,R_p)
              / (ndeg_e(R_e) ndeg_p(R_p))                 (n_b x n_b per mode ka)
  g_mn,nu(k,q) = [U_{k+q}^dagger (sum_ka g_ka(k,q) e_ka,nu(q)) U_k]_mn
                 / sqrt(2 omega_q,nu)                       (Sec. 3 Eq. (2))

The last line carries the 1/sqrt(2 omega) of Eq. (2); the overlap
U_k U_{k+q}^dagger that Sec. 4 prints for the polar term is the same pair of
rotation matrices.  Atomic positions are not part of the phases (lattice
vectors only).
"""
import numpy as np


def phases(points, R, ndeg):
    """exp(2 pi i p.R) / ndeg(R) for every point p and vector R.
    points [P][3] float64 fractional, R [N][3] int, ndeg [N] int ->
    [P][N] complex128.  The argument p.R is reduced to [-1/2, 1/2) before the
    exponential so large R do not lose phase accuracy."""
    x = np.asarray(points, dtype=np.float64) @ np.asarray(R, dtype=np.float64).T
    x = x - np.floor(x + 0.5)
    return np.exp(2j * np.pi * x) / np.asarray(ndeg, dtype=np.float64)[None, :]


def interpolate(XR, R, ndeg, points):
    """X(p) = sum_R exp(2 pi i p.R) X(R)/ndeg(R); XR [N][...] -> [P][...]."""
    XR = np.asarray(XR)
    ph = phases(points, R, ndeg)
    flat = XR.reshape(XR.shape[0], -1).astype(np.complex128)
    return (ph @ flat).reshape((len(points),) + XR.shape[1:])


def hermitise(M):
    """(M + M^dagger)/2 over the last two axes."""
    return 0.5 * (M + np.conj(np.swapaxes(M, -1, -2)))


def bands(HR, R, ndeg, kpoints):
    """Band energies eps[P][nb] (ascending) and eigenvectors U[P][nb][nb]
    (columns) of the interpolated, Hermitised H(k)."""
    Hk = hermitise(interpolate(HR, R, ndeg, kpoints))
    eps, U = np.linalg.eigh(Hk)
    return eps, U


def phonons(DR, R, ndeg, qpoints):
    """Phonon frequencies omega[P][nm] and eigenvectors e[P][nm][nm]
    (columns) of the interpolated, Hermitised D(q).  omega = sign(l) sqrt|l|
    for each eigenvalue l of D(q), so unstable modes come out negative."""
    Dq = hermitise(interpolate(DR, R, ndeg, qpoints))
    lam, e = np.linalg.eigh(Dq)
    omega = np.sign(lam) * np.sqrt(np.abs(lam))
    return omega, e


def vertex_wannier(gR, Re, ndeg_e, Rp, ndeg_p, k, qpoints):
    """g_ka(k,q) in the Wannier basis for ONE k and all q.

    gR [Ne][Np][nm][nb][nb] -> [Q][nm][nb][nb].  The double sum over
    (R_e, R_p) is taken R_e first (k fixed), then R_p; the order is free
    because both sums are finite and exact."""
    ne, npp = gR.shape[0], gR.shape[1]
    ph_e = phases(np.asarray(k, dtype=np.float64)[None, :], Re, ndeg_e)[0]   # [Ne]
    g_k = np.tensordot(ph_e, gR, axes=(0, 0))                                # [Np][nm][nb][nb]
    ph_q = phases(qpoints, Rp, ndeg_p)                                       # [Q][Np]
    out = ph_q @ g_k.reshape(npp, -1)
    return out.reshape((len(qpoints),) + gR.shape[2:])


def rotate(gw, U_k, U_kq, e_q, omega_q, omega_cut):
    """Rotate Wannier-basis g into the band/mode basis (Sec. 3 Eq. (2)).

    gw [Q][nm][nb][nb] (Cartesian modes ka, rows = k+q side, cols = k side),
    U_k [nb][nb], U_kq [Q][nb][nb], e_q [Q][nm][nm], omega_q [Q][nm].
    Returns g[Q][nu][m][n] = [U_kq^dag (sum_ka gw_ka e_ka,nu) U_k]_mn /
    sqrt(2 omega_nu), set to 0 for modes with omega < omega_cut."""
    gmode = np.einsum("qaij,qav->qvij", gw, e_q)
    gband = np.einsum("qim,qvij,jn->qvmn", np.conj(U_kq), gmode, U_k)
    keep = omega_q >= omega_cut
    scale = np.zeros_like(omega_q)
    scale[keep] = 1.0 / np.sqrt(2.0 * omega_q[keep])
    return gband * scale[:, :, None, None]
