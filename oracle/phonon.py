"""Phonon linewidth (Sec. 3 Eq. (9)) and the mode-resolved electron-phonon
coupling strength lambda_q,nu (Sec. 3 Eq. (11)), oracle side.

Test infrastructure only (see oracle/__init__.py).

  Pi''_q,nu = (2 pi / N_k) sum_k sum_mn |g_mn,nu(k,q)|^2
                 [f_nk - f_m,k+q] delta(eps_nk - eps_m,k+q - omega)

  lambda_q,nu = 1 / (N(eps_F) omega_q,nu) (1 / N_k) sum_k sum_mn |g_mn,nu(k,q)|^2
                 delta(eps_nk - eps_F) delta(eps_m,k+q - eps_F)

  N(eps_F) = (1 / N_k) sum_nk delta(eps_nk - eps_F)   (density of states per spin)

Readings of the paper taken here (listed with their reasons in the design
notes):
  * the phonon linewidth is evaluated on shell, omega = omega_q,nu; the sign
    follows the printed delta argument, so for omega > 0 the value is the
    (non-positive) imaginary part of the retarded self-energy and the
    linewidth is its magnitude;
  * the BZ integral over k becomes (1/N_k) sum_k over the given k set, and
    N(eps_F) is taken on the same set with the same Gaussian delta_sigma as
    the self-energy; lambda is 0 where N(eps_F) = 0;
  * eps_F = mu; f is Fermi-Dirac at T (as for Eq. (8));
  * modes with omega < omega_cut give 0 (as for Eq. (8));
  * degenerate modes: both quantities are averaged over modes of one q whose
    sorted frequencies differ by less than deg_tol, which makes them
    independent of the eigenvector choice inside a degenerate subspace (the
    sums over m and n already run over complete band sets).
"""
import numpy as np

from . import interp
from .selfenergy import degenerate_average, fermi, gaussian


def phonon_sums_one_k(gband, eps_k, eps_kq, omega_q, mu, T, sigma, omega_cut=1e-3):
    """The k-th terms of the two sums, for ONE k and all q.
    gband [Q][nu][m][n], eps_k [nb] (band n at k), eps_kq [Q][nb] (band m at
    k+q), omega_q [Q][nm].  Returns (P [Q][nu], L [Q][nu]) with
      P = sum_mn |g|^2 [f_nk - f_m,k+q] delta(eps_nk - eps_m,k+q - omega_q,nu)
      L = sum_mn |g|^2 delta(eps_nk - mu) delta(eps_m,k+q - mu)
    and 0 for modes with omega < omega_cut."""
    keep = omega_q >= omega_cut
    amp = np.abs(gband) ** 2                                        # [Q][nu][m][n]
    fn = fermi(eps_k, mu, T)[None, None, None, :]
    fm = fermi(eps_kq, mu, T)[:, None, :, None]
    x = eps_k[None, None, None, :] - eps_kq[:, None, :, None] - omega_q[:, :, None, None]
    P = np.sum(amp * (fn - fm) * gaussian(x, sigma), axis=(2, 3))
    dn = gaussian(eps_k - mu, sigma)[None, None, None, :]
    dm = gaussian(eps_kq - mu, sigma)[:, None, :, None]
    L = np.sum(amp * dn * dm, axis=(2, 3))
    return P * keep, L * keep


def dos_at_fermi(eps, mu, sigma):
    """N(eps_F) per spin on the given set: (1/N_k) sum_nk delta_sigma(eps_nk - mu)."""
    eps = np.asarray(eps, dtype=np.float64)
    return float(np.sum(gaussian(eps - mu, sigma))) / eps.shape[0]


def phonon_selfenergy(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, kpoints, qpoints, T, mu, sigma,
                      omega_cut=1e-3, deg_tol=1e-6, kq_points=None, phonon_states=None, loop="k"):
    """(Pi'' [Nq][nm], lambda [Nq][nm]) for the given k and q points.

    Every step is a direct evaluation, as in selfenergy.imsigma: bands at k
    and at k+q, phonons at q, the Wannier-basis vertex per k, the rotation of
    Eq. (2), the two sums over m, n and k, the normalisations, then the
    average over degenerate modes.  kq_points and phonon_states as in
    selfenergy.imsigma.  loop="q" takes the q points one at a time with all
    k at once (the vertex summed over R_p first): the same sums in another
    order, for few q and many k (kq_points is not used there)."""
    kpoints = np.asarray(kpoints, dtype=np.float64)
    qpoints = np.asarray(qpoints, dtype=np.float64)
    if loop == "q":
        return _phonon_selfenergy_by_q(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, kpoints, qpoints, T, mu, sigma,
                                       omega_cut, deg_tol, phonon_states)
    nk = len(kpoints)
    eps_k, U_k = interp.bands(HR, Re, ndeg_e, kpoints)
    if phonon_states is None:
        omega, evec = interp.phonons(DR, Rp, ndeg_p, qpoints)
    else:
        omega, evec = phonon_states
    P = np.zeros(omega.shape)
    L = np.zeros(omega.shape)
    for ik, k in enumerate(kpoints):
        kq = k[None, :] + qpoints if kq_points is None else kq_points[ik]
        eps_kq, U_kq = interp.bands(HR, Re, ndeg_e, kq)
        gw = interp.vertex_wannier(gR, Re, ndeg_e, Rp, ndeg_p, k, qpoints)
        gb = interp.rotate(gw, U_k[ik], U_kq, evec, omega, omega_cut)
        p, l = phonon_sums_one_k(gb, eps_k[ik], eps_kq, omega, mu, T, sigma, omega_cut)
        P += p
        L += l
    pi_im = (2.0 * np.pi / nk) * P
    dos = dos_at_fermi(eps_k, mu, sigma)
    keep = omega >= omega_cut
    lam = np.zeros(omega.shape)
    if dos > 0.0:
        lam[keep] = L[keep] / (nk * dos * omega[keep])
    return (degenerate_average(omega, pi_im, deg_tol), degenerate_average(omega, lam, deg_tol))


def _phonon_selfenergy_by_q(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, kpoints, qpoints, T, mu, sigma,
                            omega_cut, deg_tol, phonon_states):
    nk = len(kpoints)
    eps_k, U_k = interp.bands(HR, Re, ndeg_e, kpoints)
    if phonon_states is None:
        omega, evec = interp.phonons(DR, Rp, ndeg_p, qpoints)
    else:
        omega, evec = phonon_states
    ne, npp = gR.shape[0], gR.shape[1]
    ph_k = interp.phases(kpoints, Re, ndeg_e)                                 # [Nk][Ne]
    P = np.zeros(omega.shape)
    L = np.zeros(omega.shape)
    for iq, q in enumerate(qpoints):
        ph_q = interp.phases(q[None, :], Rp, ndeg_p)[0]                       # [Np]
        g_eq = np.tensordot(ph_q, gR, axes=(0, 1))                            # [Ne][nm][nb][nb]
        gw = (ph_k @ g_eq.reshape(ne, -1)).reshape((nk,) + gR.shape[2:])      # [Nk][nm][nb][nb]
        eps_kq, U_kq = interp.bands(HR, Re, ndeg_e, kpoints + q[None, :])
        # Eq. (2) for every k at this q: [U_k+q^dag (sum_a g_a e_a,nu) U_k] / sqrt(2 omega)
        w = omega[iq]
        keep = w >= omega_cut
        scale = np.where(keep, 1.0 / np.sqrt(2.0 * np.where(keep, w, 1.0)), 0.0)
        gmode = np.einsum("kaij,av->kvij", gw, evec[iq])
        gb = np.einsum("kim,kvij,kjn->kvmn", np.conj(U_kq), gmode, U_k, optimize=True) * scale[None, :, None, None]
        amp = np.abs(gb) ** 2                                                 # [Nk][nu][m][n]
        fn = fermi(eps_k, mu, T)[:, None, None, :]
        fm = fermi(eps_kq, mu, T)[:, None, :, None]
        x = eps_k[:, None, None, :] - eps_kq[:, None, :, None] - w[None, :, None, None]
        P[iq] = np.sum(amp * (fn - fm) * gaussian(x, sigma), axis=(0, 2, 3)) * keep
        dn = gaussian(eps_k - mu, sigma)[:, None, None, :]
        dm = gaussian(eps_kq - mu, sigma)[:, None, :, None]
        L[iq] = np.sum(amp * dn * dm, axis=(0, 2, 3)) * keep
    pi_im = (2.0 * np.pi / nk) * P
    dos = dos_at_fermi(eps_k, mu, sigma)
    keep = omega >= omega_cut
    lam = np.zeros(omega.shape)
    if dos > 0.0:
        lam[keep] = L[keep] / (nk * dos * omega[keep])
    return (degenerate_average(omega, pi_im, deg_tol), degenerate_average(omega, lam, deg_tol))
