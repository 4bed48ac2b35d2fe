"""Real part of the electron self-energy (Sec. 3 Eq. (3)) on shell and its
Fermi-level-referenced form (Sec. 3 Eq. (5)), oracle side.

Test infrastructure only (see oracle/__init__.py).

  Sigma'_nk(omega) = (1 / N_q) sum_q sum_m,nu |g_mn,nu(k,q)|^2 Re{
        [n_q,nu + f_m,k+q] / (omega - (eps_m,k+q - eps_F) + omega_q,nu + i delta)
      + [n_q,nu + 1 - f_m,k+q] / (omega - (eps_m,k+q - eps_F) - omega_q,nu + i delta) }

  with Re 1/(x + i delta) = x / (x^2 + delta^2), and

  Sigma~'_nk = Sigma'_nk(omega = eps_nk - eps_F) - Sigma'_nk(omega = 0)      (Eq. (5))

Readings of the paper taken here (listed with their reasons in the design
notes): omega is taken on shell, omega = eps_nk - eps_F (as for Eq. (8)),
and omega = eps_F in the subtracted term is omega = 0 on that scale; the
small positive delta of Eq. (3) is the broadening sigma of the run; eps_F =
mu; the occupations, the BZ mean, omega_cut and the degenerate average are
those of Eq. (8).
"""
import numpy as np

from . import interp
from .selfenergy import bose, degenerate_average, fermi


def resigma_terms(eps_k, eps_kq, omega_q, mu, T, delta, at):
    """The real part of the bracket of Eq. (3) for every (q, nu, m, n) at
    omega = eps_nk - mu (at="shell") or omega = 0 (at="fermi").
    eps_k [nb], eps_kq [Q][nb], omega_q [Q][nm] -> [Q][nu][m][n]."""
    nq = bose(omega_q, T)[:, :, None, None]
    f = fermi(eps_kq, mu, T)[:, None, :, None]
    w = omega_q[:, :, None, None]
    om = (eps_k - mu) if at == "shell" else np.zeros_like(eps_k)
    base = om[None, None, None, :] - (eps_kq - mu)[:, None, :, None]
    x1, x2 = base + w, base - w
    return (nq + f) * x1 / (x1 * x1 + delta * delta) + (nq + 1.0 - f) * x2 / (x2 * x2 + delta * delta)


def resigma_from_states(gband, eps_k, eps_kq, omega_q, mu, T, delta, nq_norm, omega_cut=1e-3):
    """(Sigma'_nk(eps_nk - mu), Sigma'_nk(0)) for one k from band/mode-basis
    vertices gband [Q][nu][m][n] (before the degenerate average)."""
    keep = omega_q >= omega_cut
    safe = np.where(keep, omega_q, 1.0)
    amp = np.abs(gband) ** 2 * keep[:, :, None, None]
    shell = np.sum(amp * resigma_terms(eps_k, eps_kq, safe, mu, T, delta, "shell"), axis=(0, 1, 2))
    fermi0 = np.sum(amp * resigma_terms(eps_k, eps_kq, safe, mu, T, delta, "fermi"), axis=(0, 1, 2))
    return shell / nq_norm, fermi0 / nq_norm


def resigma(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, kpoints, qpoints, T, mu, delta,
            omega_cut=1e-3, deg_tol=1e-6, nq_norm=None, phonon_states=None):
    """(Sigma'_nk on shell [Nk][nb], Sigma~'_nk [Nk][nb]) in eV: the same
    direct evaluation as selfenergy.imsigma (bands at k and k+q, phonons,
    vertex per k, rotation of Eq. (2)) with the real-part weights, then the
    degenerate average of both."""
    kpoints = np.asarray(kpoints, dtype=np.float64)
    qpoints = np.asarray(qpoints, dtype=np.float64)
    if nq_norm is None:
        nq_norm = len(qpoints)
    eps_k, U_k = interp.bands(HR, Re, ndeg_e, kpoints)
    if phonon_states is None:
        omega, evec = interp.phonons(DR, Rp, ndeg_p, qpoints)
    else:
        omega, evec = phonon_states
    nb = eps_k.shape[1]
    shell = np.zeros((len(kpoints), nb))
    fermi0 = np.zeros((len(kpoints), nb))
    for ik, k in enumerate(kpoints):
        eps_kq, U_kq = interp.bands(HR, Re, ndeg_e, k[None, :] + qpoints)
        gw = interp.vertex_wannier(gR, Re, ndeg_e, Rp, ndeg_p, k, qpoints)
        gb = interp.rotate(gw, U_k[ik], U_kq, evec, omega, omega_cut)
        shell[ik], fermi0[ik] = resigma_from_states(gb, eps_k[ik], eps_kq, omega, mu, T, delta, nq_norm,
                                                    omega_cut)
    shell = degenerate_average(eps_k, shell, deg_tol)
    fermi0 = degenerate_average(eps_k, fermi0, deg_tol)
    return shell, shell - fermi0
