"""Complex electron self-energy Sigma_nk(omega) on a frequency grid (Sec. 3
Eq. (3)), its Fermi-level-referenced real part (Sec. 3 Eq. (5)) and the
electronic spectral function A_nk(omega) (Sec. 3 Eq. (10)), oracle side.

Test infrastructure only (see oracle/__init__.py).

  Sigma_nk(omega) = (1 / N_q) sum_q sum_m,nu |g_mn,nu(k,q)|^2 {
        [n_q,nu + f_m,k+q] / (omega - (eps_m,k+q - eps_F) + omega_q,nu + i delta)
      + [n_q,nu + 1 - f_m,k+q] / (omega - (eps_m,k+q - eps_F) - omega_q,nu + i delta) }

  Sigma~'_nk(omega) = Re Sigma_nk(omega) - Re Sigma_nk(0)                 (Eq. (5))

  A_nk(omega) = (1/pi) |Sigma''| / ( (omega - (eps_nk - eps_F) - Sigma~')^2 + Sigma''^2 )

Readings of the paper taken here (listed with their reasons in the design
notes): omega is measured from eps_F, as in the denominators of Eq. (3), so
"omega = eps_F" of Eq. (5) is omega = 0; delta is the run's broadening
sigma; Sigma'' in Eq. (10) is the imaginary part of the same Eq. (3) at the
same finite delta (a Lorentzian delta; it tends to Eq. (8) as delta -> 0), so
that Sigma' and Sigma'' are the two parts of one retarded function; the
denominator of Eq. (10) adds Sigma''^2 (printed without the square, which is
not dimensionally consistent and would not give a normalised spectral
function); eps_F = mu; occupations, omega_cut, the BZ mean and the degenerate
average as for Eq. (8).
"""
import numpy as np

from . import interp
from .selfenergy import bose, degenerate_average, fermi


def bracket(eps_kq, omega_q, mu, T, delta, wgrid):
    """The braces of Eq. (3) as complex numbers for every (q, nu, m, omega).
    eps_kq [Q][nb] (band m at k+q), omega_q [Q][nm], wgrid [W]
    -> [Q][nu][m][W].  The braces do not depend on the band n at k."""
    nq = bose(omega_q, T)[:, :, None, None]
    f = fermi(eps_kq, mu, T)[:, None, :, None]
    w = omega_q[:, :, None, None]
    xi = (eps_kq - mu)[:, None, :, None]
    om = np.asarray(wgrid, dtype=np.float64)[None, None, None, :]
    return (nq + f) / (om - xi + w + 1j * delta) + (nq + 1.0 - f) / (om - xi - w + 1j * delta)


def sigma_from_states(gband, eps_kq, omega_q, mu, T, delta, wgrid, nq_norm, omega_cut=1e-3):
    """Sigma_n(omega) [nb][W] (complex) for one k from band/mode-basis
    vertices gband [Q][nu][m][n], before the degenerate average."""
    keep = omega_q >= omega_cut
    safe = np.where(keep, omega_q, 1.0)
    amp = np.abs(gband) ** 2 * keep[:, :, None, None]                   # [Q][nu][m][n]
    br = bracket(eps_kq, safe, mu, T, delta, wgrid)                    # [Q][nu][m][W]
    return np.einsum("qvmn,qvmw->nw", amp, br) / nq_norm


def selfenergy_omega(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, kpoints, qpoints, T, mu, delta, wgrid,
                     omega_cut=1e-3, deg_tol=1e-6, nq_norm=None, phonon_states=None):
    """(Sigma [Nk][nb][W] complex, Sigma(omega = 0) [Nk][nb] complex, eps_k
    [Nk][nb]): bands at k and k+q, phonons at q, the Wannier-basis vertex per
    k, the rotation of Eq. (2), the sum of Eq. (3) over q, m and nu, then the
    average over degenerate bands at every omega."""
    kpoints = np.asarray(kpoints, dtype=np.float64)
    qpoints = np.asarray(qpoints, dtype=np.float64)
    wgrid = np.asarray(wgrid, dtype=np.float64)
    if nq_norm is None:
        nq_norm = len(qpoints)
    eps_k, U_k = interp.bands(HR, Re, ndeg_e, kpoints)
    if phonon_states is None:
        omega, evec = interp.phonons(DR, Rp, ndeg_p, qpoints)
    else:
        omega, evec = phonon_states
    nb = eps_k.shape[1]
    wall = np.concatenate([wgrid, [0.0]])
    sig = np.zeros((len(kpoints), nb, len(wall)), dtype=np.complex128)
    for ik, k in enumerate(kpoints):
        eps_kq, U_kq = interp.bands(HR, Re, ndeg_e, k[None, :] + qpoints)
        gw = interp.vertex_wannier(gR, Re, ndeg_e, Rp, ndeg_p, k, qpoints)
        gb = interp.rotate(gw, U_k[ik], U_kq, evec, omega, omega_cut)
        sig[ik] = sigma_from_states(gb, eps_kq, omega, mu, T, delta, wall, nq_norm, omega_cut)
    for iw in range(len(wall)):
        sig[:, :, iw] = (degenerate_average(eps_k, sig[:, :, iw].real, deg_tol)
                         + 1j * degenerate_average(eps_k, sig[:, :, iw].imag, deg_tol))
    return sig[:, :, :-1], sig[:, :, -1], eps_k


def spectral_function(eps_k, mu, wgrid, sigma_w, sigma0):
    """A_nk(omega) of Eq. (10) [Nk][nb][W] from Sigma_nk(omega) [Nk][nb][W]
    and Sigma_nk(0) [Nk][nb] (complex), with Sigma~' of Eq. (5)."""
    w = np.asarray(wgrid, dtype=np.float64)[None, None, :]
    tilde = sigma_w.real - np.asarray(sigma0).real[:, :, None]
    im = np.abs(sigma_w.imag)
    den = (w - (np.asarray(eps_k) - mu)[:, :, None] - tilde) ** 2 + im ** 2
    return im / (np.pi * den)
