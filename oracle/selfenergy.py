"""Imaginary electron self-energy (linewidth) of Sec. 3 Eq. (8), oracle side.

Test infrastructure only (see oracle/__init__.py).

  Im Sigma_nk = (pi / N_q) sum_q sum_m sum_nu |g_mn,nu(k,q)|^2
      { [n_q,nu + f_m,k+q] delta(eps_nk - eps_m,k+q + omega_q,nu)
      + [n_q,nu + 1 - f_m,k+q] delta(eps_nk - eps_m,k+q - omega_q,nu) }

Readings of the paper taken here (each one listed with its reason in the
design notes):
  * the BZ integral over q with weight dq/Omega_BZ becomes the uniform mean
    (1/N_q) sum_q, for grids and for random points alike (Sec. 10.1, 10.2);
  * the self-energy is evaluated on shell, omega = eps_nk - eps_F, so the
    delta arguments are eps_nk - eps_m,k+q +- omega_q,nu and eps_F = mu
    enters only the Fermi function;
  * n(omega) = 1/(exp(omega/k_B T) - 1) (defined under Eq. (4)); f is the
    Fermi-Dirac function at the same T (the paper does not spell f out);
  * the delta function is a Gaussian of width sigma,
    delta_sigma(x) = exp(-x^2/sigma^2) / (sigma sqrt(pi))  (Sec. 10.1, 10.2
    use Gaussian broadening without fixing the width convention);
  * units: eV for energies, K for T, hbar = 1;
  * degenerate states: Im Sigma is averaged over bands whose sorted
    eigenvalues differ by less than deg_tol (gauge invariance by averaging
    over degenerate states, Sec. 10.4).
"""
import numpy as np

from . import interp

KB_EV = 8.617333262e-5   # Boltzmann constant in eV/K (CODATA 2018)


def fermi(eps, mu, T):
    """Fermi-Dirac occupation; T = 0 gives the step with 1/2 at eps = mu."""
    eps = np.asarray(eps, dtype=np.float64)
    if T == 0.0:
        return np.where(eps < mu, 1.0, np.where(eps > mu, 0.0, 0.5))
    x = (eps - mu) / (KB_EV * T)
    with np.errstate(over="ignore"):
        return 1.0 / (np.exp(x) + 1.0)


def bose(omega, T):
    """Bose-Einstein occupation 1/(exp(omega/k_B T) - 1); 0 at T = 0."""
    omega = np.asarray(omega, dtype=np.float64)
    if T == 0.0:
        return np.zeros_like(omega)
    with np.errstate(over="ignore", divide="ignore"):
        return 1.0 / np.expm1(omega / (KB_EV * T))


def gaussian(x, sigma):
    """Normalised Gaussian delta_sigma(x) = exp(-x^2/sigma^2)/(sigma sqrt pi)."""
    x = np.asarray(x, dtype=np.float64)
    return np.exp(-(x / sigma) ** 2) / (sigma * np.sqrt(np.pi))


def weights(eps_k, eps_kq, omega_q, mu, T, sigma):
    """The curly bracket of Eq. (8) for every (q, nu, m, n):
    eps_k [nb] (band n at k), eps_kq [Q][nb] (band m at k+q), omega_q [Q][nm].
    Returns W[Q][nu][m][n]."""
    nq = bose(omega_q, T)[:, :, None, None]                 # [Q][nu][1][1]
    f = fermi(eps_kq, mu, T)[:, None, :, None]              # [Q][1][m][1]
    x = eps_k[None, None, None, :] - eps_kq[:, None, :, None]
    w = omega_q[:, :, None, None]
    return (nq + f) * gaussian(x + w, sigma) + (nq + 1.0 - f) * gaussian(x - w, sigma)


def degenerate_average(eps, values, deg_tol):
    """Average values[P][nb] over groups of bands whose consecutive sorted
    energies eps[P][nb] differ by less than deg_tol."""
    out = np.array(values, dtype=np.float64, copy=True)
    for p in range(eps.shape[0]):
        start = 0
        nb = eps.shape[1]
        while start < nb:
            stop = start + 1
            while stop < nb and abs(eps[p, stop] - eps[p, stop - 1]) < deg_tol:
                stop += 1
            out[p, start:stop] = np.mean(values[p, start:stop])
            start = stop
    return out


def imsigma_from_states(gband, eps_k, eps_kq, omega_q, mu, T, sigma, nq_norm,
                        omega_cut=1e-3):
    """Eq. (8) for one k from band/mode-basis vertices.
    gband [Q][nu][m][n], eps_k [nb], eps_kq [Q][nb], omega_q [Q][nm].
    Modes with omega < omega_cut contribute nothing (their Bose factor may
    be infinite at omega = 0).  Returns Im Sigma[nb] before the degenerate
    average; nq_norm is the N_q of the BZ mean."""
    keep = omega_q >= omega_cut
    safe = np.where(keep, omega_q, 1.0)
    W = weights(eps_k, eps_kq, safe, mu, T, sigma)
    W = W * keep[:, :, None, None]
    return (np.pi / nq_norm) * np.sum(np.abs(gband) ** 2 * W, axis=(0, 1, 2))


def imsigma(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, kpoints, qpoints, T, mu, sigma,
            omega_cut=1e-3, deg_tol=1e-6, nq_norm=None, kq_points=None,
            phonon_states=None):
    """Im Sigma_nk [Nk][nb] (eV) of Eq. (8) for the given k and q points.

    Every step is a direct evaluation: interpolation and eigensolves at k, at
    q and at k+q (the unfolded sum k+q: exp(2 pi i G.R) = 1 makes it equal
    to the folded grid point), the Wannier-basis vertex per k, the rotation of
    Eq. (2), the weights of Eq. (8), then the degenerate average.
    kq_points, when given ([Nk][Nq][3]), replaces k+q (used by tests that pin
    the k+q convention); phonon_states=(omega [Nq][nm], e [Nq][nm][nm]), when
    given, replaces the interpolated phonons (the frequencies are then an
    input, as for the gradient with respect to omega)."""
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
    out = np.zeros((len(kpoints), nb))
    for ik, k in enumerate(kpoints):
        kq = k[None, :] + qpoints if kq_points is None else kq_points[ik]
        eps_kq, U_kq = interp.bands(HR, Re, ndeg_e, kq)
        gw = interp.vertex_wannier(gR, Re, ndeg_e, Rp, ndeg_p, k, qpoints)
        gb = interp.rotate(gw, U_k[ik], U_kq, evec, omega, omega_cut)
        out[ik] = imsigma_from_states(gb, eps_k[ik], eps_kq, omega, mu, T, sigma, nq_norm,
                                      omega_cut)
    return degenerate_average(eps_k, out, deg_tol)
