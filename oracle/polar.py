"""Long-range (polar) part of the electron-phonon vertex, Sec. 4, oracle side.

Test infrastructure only (see oracle/__init__.py).

  g_mn,nu(k,q) = g^S_mn,nu(k,q) + g^L_mn,nu(k,q)                      (Sec. 4)

  g^L_mn,nu(k,q) = L_nu(q) [U_k+q^dagger U_k]_mn

  L_nu(q) = i C sum_kappa (1 / (2 M_kappa omega_q,nu))^(1/2)
              sum_{G, q+G != 0} exp(-K.eps.K / (4 alpha)) / (K.eps.K)
              (K . Z*_kappa . e_kappa,nu(q)) exp(-i K . tau_kappa),   K = q + G

The short-range g^S is the Wannier interpolation of the rest of the oracle
(interp.vertex_wannier + interp.rotate); the long-range part is added to it
for every (k, q), as in step (iv) of the paper's scheme.

Readings of the paper taken here (listed with their reasons in the design
notes):
  * the overlap <psi_m,k+q| exp(i(q+G).r) |psi_nk> in the small-(q+G) form
    the paper prints is the Wannier-gauge overlap [U_k+q^dagger U_k]_mn with
    U columns = bands (the paper writes the same product with rows = bands);
  * the G sum, which the printed equation leaves unbounded, carries the
    Gaussian factor exp(-K.eps.K / (4 alpha)) of the method the paper cites,
    with alpha a run parameter; terms with K.eps.K / (4 alpha) >= cutoff are
    dropped (each below exp(-cutoff) of the leading one);
  * the phase exp(-i K . tau_kappa) of an atom at tau_kappa in the cell, absent
    from the printed equation and required by the lattice-vector phase
    convention of the interpolation (the dipole of atom kappa in cell R sits
    at R + tau_kappa);
  * C is the overall factor (4 pi e^2 / Omega in the run's units), which the
    printed equation omits; hbar = 1;
  * e_q,nu are eigenvectors of the mass-scaled dynamical matrix (the masses
    are folded into the modes) and M_kappa enters only through the explicit
    (1 / (2 M omega))^(1/2);
  * modes with omega < omega_cut give 0, as everywhere else.
"""
import itertools

import numpy as np

from . import interp


def reciprocal_vectors(vectors):
    """Rows b_i with a_i . b_j = 2 pi delta_ij for primitive rows a_i."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(vectors, dtype=np.float64)).T


def _gmax(vectors, eps_inf, alpha, cutoff):
    """Half-width of a box of integer G coordinates that holds every K = q + G
    with K.eps.K / (4 alpha) < cutoff for any q in the first cell (q reduced
    to [-1/2, 1/2)^3)."""
    A = np.asarray(vectors, dtype=np.float64)
    B = reciprocal_vectors(A)
    lam_min = np.linalg.eigvalsh(np.asarray(eps_inf, dtype=np.float64)).min()
    kmax = np.sqrt(4.0 * alpha * cutoff / lam_min)
    qmax = 0.5 * np.abs(B).sum()
    return int(np.ceil(np.max(np.linalg.norm(A, axis=1)) * (kmax + qmax) / (2.0 * np.pi))) + 1


def long_range_factor(qpoints, omega, evec, vectors, tau, zstar, eps_inf, masses, prefactor, alpha, cutoff,
                      omega_cut=1e-3, gmax=None):
    """L_nu(q) [Q][nm] complex: the long-range vertex before the overlap.
    qpoints [Q][3] fractional; omega [Q][nm]; evec [Q][nm][nm] (columns,
    row index 3 kappa + Cartesian direction); vectors [3][3] primitive rows
    (Cartesian); tau [nat][3] Cartesian; zstar [nat][3][3]; eps_inf [3][3];
    masses [nat].  gmax overrides the G box half-width."""
    q = np.asarray(qpoints, dtype=np.float64)
    B = reciprocal_vectors(vectors)
    eps_inf = np.asarray(eps_inf, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    zstar = np.asarray(zstar, dtype=np.float64)
    masses = np.asarray(masses, dtype=np.float64)
    nat = len(tau)
    nm = omega.shape[1]
    g = _gmax(vectors, eps_inf, alpha, cutoff) if gmax is None else gmax
    grid = np.array(list(itertools.product(range(-g, g + 1), repeat=3)), dtype=np.float64)
    out = np.zeros((len(q), nm), dtype=np.complex128)
    for iq in range(len(q)):
        qr = q[iq] - np.floor(q[iq] + 0.5)              # the sum over all G is periodic in q
        K = (qr[None, :] + grid) @ B                    # [nG][3] Cartesian
        x = np.einsum("ga,ab,gb->g", K, eps_inf, K)
        use = (np.einsum("ga,ga->g", K, K) > 1e-24) & (x / (4.0 * alpha) < cutoff)
        K, x = K[use], x[use]
        f = np.exp(-x / (4.0 * alpha)) / x              # [nG]
        acc = np.zeros(nm, dtype=np.complex128)
        for kap in range(nat):
            zK = K @ zstar[kap]                          # (K . Z*_kappa)_b   [nG][3]
            e_k = evec[iq, 3 * kap:3 * kap + 3, :]       # [3][nm]
            ph = np.exp(-1j * (K @ tau[kap]))            # [nG]
            acc += np.einsum("g,g,gb,bv->v", f, ph, zK, e_k) / np.sqrt(masses[kap])
        keep = omega[iq] >= omega_cut
        sc = np.where(keep, 1.0 / np.sqrt(2.0 * np.where(keep, omega[iq], 1.0)), 0.0)
        out[iq] = 1j * prefactor * sc * acc
    return out


def vertex_band(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, k, qpoints, polar, omega_cut=1e-3, phonon_states=None,
                lr=None):
    """(g [Q][nu][m][n] = g^S + g^L for ONE k and all q, eps_k [nb], eps_kq [Q][nb],
    omega [Q][nm]).  polar: dict(vectors, tau, zstar, eps_inf, masses,
    prefactor, alpha, cutoff); lr, when given, is L_nu(q) for these q
    (it does not depend on k)."""
    k = np.asarray(k, dtype=np.float64)
    qpoints = np.asarray(qpoints, dtype=np.float64)
    eps_k, U_k = interp.bands(HR, Re, ndeg_e, k[None, :])
    eps_kq, U_kq = interp.bands(HR, Re, ndeg_e, k[None, :] + qpoints)
    if phonon_states is None:
        omega, evec = interp.phonons(DR, Rp, ndeg_p, qpoints)
    else:
        omega, evec = phonon_states
    gw = interp.vertex_wannier(gR, Re, ndeg_e, Rp, ndeg_p, k, qpoints)
    gS = interp.rotate(gw, U_k[0], U_kq, evec, omega, omega_cut)
    L = long_range_factor(qpoints, omega, evec, omega_cut=omega_cut, **polar) if lr is None else lr
    ov = np.einsum("qim,in->qmn", np.conj(U_kq), U_k[0])          # [U_k+q^dag U_k]_mn
    return gS + L[:, :, None, None] * ov[:, None, :, :], eps_k[0], eps_kq, omega


def imsigma(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, kpoints, qpoints, T, mu, sigma, polar,
            omega_cut=1e-3, deg_tol=1e-6, nq_norm=None):
    """Im Sigma_nk of Sec. 3 Eq. (8) with the polar vertex g^S + g^L (the
    phonons and L_nu(q) are evaluated once for all k)."""
    from .selfenergy import degenerate_average, imsigma_from_states
    kpoints = np.asarray(kpoints, dtype=np.float64)
    qpoints = np.asarray(qpoints, dtype=np.float64)
    if nq_norm is None:
        nq_norm = len(qpoints)
    eps_all, _ = interp.bands(HR, Re, ndeg_e, kpoints)
    ph = interp.phonons(DR, Rp, ndeg_p, qpoints)
    L = long_range_factor(qpoints, ph[0], ph[1], omega_cut=omega_cut, **polar)
    out = np.zeros(eps_all.shape)
    for ik, k in enumerate(kpoints):
        g, ek, ekq, om = vertex_band(HR, Re, ndeg_e, DR, Rp, ndeg_p, gR, k, qpoints, polar, omega_cut,
                                     phonon_states=ph, lr=L)
        out[ik] = imsigma_from_states(g, ek, ekq, om, mu, T, sigma, nq_norm, omega_cut)
    return degenerate_average(eps_all, out, deg_tol)
