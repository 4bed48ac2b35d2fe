"""Transport coupling of Sec. 6: band velocities from the Wannier Hamiltonian
(Sec. 7), the mode-resolved transport coupling strength lambda_tr,q,nu
(Eq. (55)), the Eliashberg function alpha^2 F(omega) (Eq. (12); Eq. (54) for
the transport variant) and the Ziman resistivity integral (Eq. (53)), oracle
side.

Test infrastructure only (see oracle/__init__.py).

  v_nk,a = d eps_nk / d k_a  = Re [U_k^dagger (dH/dk_a) U_k]_nn,
      dH/dk_a = sum_R i R_a exp(2 pi i k.R) H(R) / ndeg(R)   (R Cartesian, k in 1/length)

  lambda_tr,q,nu = 1 / (N(eps_F) omega_q,nu) (1/N_k) sum_k sum_mn |g_mn,nu(k,q)|^2
      delta(eps_nk - eps_F) delta(eps_m,k+q - eps_F) (1 - v_nk . v_m,k+q / |v_nk|^2)

  alpha^2 F(omega) = (1/2) (1/N_q) sum_q,nu omega_q,nu lambda_q,nu delta(omega - omega_q,nu)

  rho(T) n e^2 / m_e = (4 pi / (k_B T)) int_0^inf d omega omega alpha_tr^2 F(omega) n(omega) [1 + n(omega)]

Readings of the paper taken here (listed with their reasons in the design
notes): the velocities are the analytic derivatives of the interpolated bands
(the Wannier route Sec. 6 and 7 name for future work; the local
approximation of Eq. (59) needs plane-wave coefficients), taken as the diagonal of the
velocity matrix and averaged over degenerate bands (the trace over a
degenerate subspace does not depend on its basis); the factor is 1 where
|v_nk|^2 <= 1e-18 (a band extremum, where it is undefined); N(eps_F), the Gaussian deltas, eps_F = mu and the degenerate-mode
average as for lambda_q,nu (Eq. (11)); alpha^2 F takes a Gaussian delta of a
given width and the BZ mean over the q set; the resistivity integral is the
trapezoid rule on the given frequency grid, hbar = 1, energies in eV.
"""
import numpy as np

from . import interp
from .phonon import dos_at_fermi
from .selfenergy import KB_EV, bose, degenerate_average, gaussian


def velocities(HR, R, ndeg, vectors, kpoints, deg_tol=1e-6):
    """v [P][nb][3] (Cartesian; eV x length) at fractional kpoints."""
    kpoints = np.asarray(kpoints, dtype=np.float64)
    Rc = np.asarray(R, dtype=np.float64) @ np.asarray(vectors, dtype=np.float64)      # [N][3]
    eps, U = interp.bands(HR, R, ndeg, kpoints)
    ph = interp.phases(kpoints, R, ndeg)                                              # [P][N]
    HRf = np.asarray(HR).reshape(len(R), -1)
    v = np.zeros(eps.shape + (3,))
    for a in range(3):
        dH = ((ph * (1j * Rc[None, :, a])) @ HRf).reshape(U.shape)
        dH = interp.hermitise(dH)
        d = np.einsum("pin,pij,pjn->pn", np.conj(U), dH, U).real
        v[:, :, a] = degenerate_average(eps, d, deg_tol)
    return v


V2_MIN = 1e-18   # |v|^2 at or below this counts as a zero velocity (band extremum)


def velocity_factor(v_n, v_m):
    """1 - v_n . v_m / |v_n|^2 for v_n [..][3], v_m [..][3]; 1 where
    |v_n|^2 <= V2_MIN (the factor is undefined at a band extremum, where the
    computed velocity is zero up to rounding)."""
    nn = np.sum(v_n * v_n, axis=-1)
    dot = np.sum(v_n * v_m, axis=-1)
    ok = nn > V2_MIN
    safe = np.where(ok, nn, 1.0)
    return np.where(ok, 1.0 - dot / safe, 1.0)


def lambda_tr(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, kpoints, qpoints, mu, sigma, vectors,
              omega_cut=1e-3, deg_tol=1e-6):
    """lambda_tr [Nq][nm] of Eq. (55), q points one at a time with all k at
    once (the vertex summed over R_p first), then the degenerate-mode average."""
    kpoints = np.asarray(kpoints, dtype=np.float64)
    qpoints = np.asarray(qpoints, dtype=np.float64)
    nk = len(kpoints)
    eps_k, U_k = interp.bands(HR, Re, ndeg_e, kpoints)
    v_k = velocities(HR, Re, ndeg_e, vectors, kpoints, deg_tol)
    omega, evec = interp.phonons(DR, Rp, ndeg_p, qpoints)
    ne = gR.shape[0]
    ph_k = interp.phases(kpoints, Re, ndeg_e)
    Lt = np.zeros(omega.shape)
    for iq, q in enumerate(qpoints):
        ph_q = interp.phases(q[None, :], Rp, ndeg_p)[0]
        g_eq = np.tensordot(ph_q, gR, axes=(0, 1))
        gw = (ph_k @ g_eq.reshape(ne, -1)).reshape((nk,) + gR.shape[2:])
        eps_kq, U_kq = interp.bands(HR, Re, ndeg_e, kpoints + q[None, :])
        v_kq = velocities(HR, Re, ndeg_e, vectors, kpoints + q[None, :], deg_tol)
        w = omega[iq]
        keep = w >= omega_cut
        scale = np.where(keep, 1.0 / np.sqrt(2.0 * np.where(keep, w, 1.0)), 0.0)
        gmode = np.einsum("kaij,av->kvij", gw, evec[iq])
        gb = np.einsum("kim,kvij,kjn->kvmn", np.conj(U_kq), gmode, U_k, optimize=True) * scale[None, :, None, None]
        amp = np.abs(gb) ** 2                                                   # [Nk][nu][m][n]
        dn = gaussian(eps_k - mu, sigma)[:, None, None, :]
        dm = gaussian(eps_kq - mu, sigma)[:, None, :, None]
        fac = velocity_factor(v_k[:, None, :, :], v_kq[:, :, None, :])          # [Nk][m][n]
        Lt[iq] = np.sum(amp * dn * dm * fac[:, None, :, :], axis=(0, 2, 3)) * keep
    dos = dos_at_fermi(eps_k, mu, sigma)
    keep = omega >= omega_cut
    lam = np.zeros(omega.shape)
    if dos > 0.0:
        lam[keep] = Lt[keep] / (nk * dos * omega[keep])
    return degenerate_average(omega, lam, deg_tol)


def eliashberg_function(omega, lam, wgrid, sigma_ph, nq_norm=None):
    """alpha^2 F(w) [W] = (1/2) (1/N_q) sum_q,nu omega lambda delta_sigma(w - omega)."""
    omega = np.asarray(omega, dtype=np.float64)
    nq = omega.shape[0] if nq_norm is None else nq_norm
    w = np.asarray(wgrid, dtype=np.float64)
    terms = (omega * lam).reshape(-1)
    return 0.5 * np.sum(terms[None, :] * gaussian(w[:, None] - omega.reshape(-1)[None, :], sigma_ph), axis=1) / nq


def ziman_integral(wgrid, a2f_tr, T):
    """(4 pi / (k_B T)) int d w  w a2F_tr(w) n(w) [1 + n(w)] by the trapezoid
    rule over the grid points with w > 0 (rho n e^2 / m_e; 0 at T = 0)."""
    if T == 0.0:
        return 0.0
    w = np.asarray(wgrid, dtype=np.float64)
    pos = w > 0.0
    n = bose(w[pos], T)
    f = np.zeros_like(w)
    f[pos] = w[pos] * np.asarray(a2f_tr)[pos] * n * (1.0 + n)
    return 4.0 * np.pi / (KB_EV * T) * np.trapezoid(f, w)
