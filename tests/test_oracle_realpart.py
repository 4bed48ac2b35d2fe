"""Pins for the oracle's on-shell real part of the electron self-energy
(Sec. 3 Eq. (3)) and its Fermi-level-referenced form (Sec. 3 Eq. (5))."""
import math

import numpy as np

from oracle import interp, lattice, realpart as rp
from paper_1604_03525_amd import inputs as I

KB = 8.617333262e-5


def _toy(kg):
    m = I.toy_model(kg, kg)
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    return R, nd, lattice.grid_points(*kg)


def _fd(e, mu, T):
    if T == 0.0:
        return 1.0 if e < mu else (0.0 if e > mu else 0.5)
    return 1.0 / (math.exp((e - mu) / (KB * T)) + 1.0)


def test_closed_form_einstein_constant_g():
    """Single band eps = -2 sum cos(2 pi k_a), Einstein phonons, constant
    g_a = c_a at R = 0: sum_nu |g_nu|^2 = sum|c|^2 / (2 omega_E) and
      Sigma'_k(w) = (sum|c|^2 / 2 omega_E) (1/N) sum_k' Re{ (n + f')/(w - xi' + omega_E + i d)
                                                          + (n + 1 - f')/(w - xi' - omega_E + i d) }
    with xi' = eps_k' - mu, written with Python complex arithmetic on the
    analytic band, at w = eps_k - mu (on shell) and w = 0."""
    kg = (6, 6, 6)
    R, nd, k = _toy(kg)
    HR = I.nn_hopping(R)
    we = 0.06
    DR = I.einstein_dynmat(R, 3, we)
    c = np.array([0.05, 0.02j, -0.03 + 0.01j])
    gR = I.constant_vertex(R, R, c)
    T, mu, d = 300.0, 0.3, 0.08
    shell, tilde = rp.resigma(HR, R, nd, DR, R, nd, gR, k, k, T, mu, d)
    eps = -2.0 * np.cos(2 * np.pi * k).sum(1)
    g2 = float(np.sum(np.abs(c) ** 2)) / (2 * we)
    n = 1.0 / math.expm1(we / (KB * T))

    def sig(w):
        s = 0.0
        for ep in eps:
            f = _fd(ep, mu, T)
            s += ((n + f) / complex(w - (ep - mu) + we, d) + (n + 1 - f) / complex(w - (ep - mu) - we, d)).real
        return g2 * s / len(eps)

    want_shell = np.array([sig(e - mu) for e in eps])
    want_f = np.array([sig(0.0) for _ in eps])
    assert np.max(np.abs(shell[:, 0] - want_shell)) < 1e-12 * np.abs(want_shell).max()
    assert np.max(np.abs(tilde[:, 0] - (want_shell - want_f))) < 1e-12 * np.abs(want_shell).max()


def test_band_bottom_moves_down_empty_band_zero_temperature():
    """T = 0, mu far below the band (every f = 0, n = 0): only the emission
    term (n + 1 - f)/(w - xi - omega + i d) remains and, for the lowest state
    (w = xi_min), its real part is negative for every q: the band bottom is
    pushed down (second-order level repulsion)."""
    R, nd, k = _toy((4, 4, 4))
    HR, DR, gR = I.toy_arrays(R, R)
    shell, tilde = rp.resigma(HR, R, nd, DR, R, nd, gR, k, k, 0.0, -10.0, 0.02)
    eps, _ = interp.bands(HR, R, nd, k)
    i0 = int(np.argmin(eps[:, 0]))
    assert shell[i0, 0] < 0.0
    # Sigma'(0) = Sigma' - Sigma~' is the same emission sum at w = 0 = eps_F,
    # far below every pole: negative for every state
    assert np.all(shell[:, 0] - tilde[:, 0] < 0.0)


def test_scaling_and_zero():
    """Sigma' and Sigma~' are quadratic in g and vanish with it."""
    R, nd, k = _toy((4, 4, 4))
    HR, DR, gR = I.toy_arrays(R, R)
    a = rp.resigma(HR, R, nd, DR, R, nd, gR, k, k, 300.0, -0.5, 0.1)
    b = rp.resigma(HR, R, nd, DR, R, nd, 1.3 * gR, k, k, 300.0, -0.5, 0.1)
    z = rp.resigma(HR, R, nd, DR, R, nd, 0.0 * gR, k, k, 300.0, -0.5, 0.1)
    for x, y, zz in zip(a, b, z):
        assert np.max(np.abs(y - 1.3 ** 2 * x)) < 1e-12 * np.abs(y).max()
        assert np.all(zz == 0.0)


def test_gauge_invariance_degenerate_blocks():
    """Two identical decoupled bands and Einstein phonons: random unitaries in
    the degenerate blocks of U_k, U_k+q and e_q leave the band-averaged
    Sigma' and Sigma~' unchanged."""
    rng = np.random.default_rng(21)
    R, nd = lattice.ws_vectors(I.SC_METRIC, (3, 3, 3))
    k = lattice.grid_points(3, 3, 3)
    h = I.nn_hopping(R)[:, 0, 0]
    HR = h[:, None, None] * np.eye(2)[None]
    DR = I.einstein_dynmat(R, 3, 0.05)
    gR = I.random_vertex(R, R, I.SC_VECTORS, 3, 2, seed=3, g0=0.1)
    T, mu, d = 300.0, 0.1, 0.2
    ref_shell, ref_tilde = rp.resigma(HR, R, nd, DR, R, nd, gR, k, k, T, mu, d)

    def haar(n):
        z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        q, r = np.linalg.qr(z)
        return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]

    eps, U = interp.bands(HR, R, nd, k)
    om, e = interp.phonons(DR, R, nd, k)
    U2 = np.einsum("pij,pjk->pik", U, np.stack([haar(2) for _ in k]))
    e2 = np.einsum("pij,pjk->pik", e, np.stack([haar(3) for _ in k]))
    shell = np.zeros((len(k), 2))
    f0 = np.zeros((len(k), 2))
    for ik, kk in enumerate(k):
        epq, Upq = interp.bands(HR, R, nd, kk[None] + k)
        Upq2 = np.einsum("pij,pjk->pik", Upq, np.stack([haar(2) for _ in k]))
        gw = interp.vertex_wannier(gR, R, nd, R, nd, kk, k)
        shell[ik], f0[ik] = rp.resigma_from_states(interp.rotate(gw, U2[ik], Upq2, e2, om, 1e-3), eps[ik], epq,
                                                   om, mu, T, d, len(k))
    from oracle.selfenergy import degenerate_average
    s2 = degenerate_average(eps, shell, 1e-6)
    t2 = s2 - degenerate_average(eps, f0, 1e-6)
    assert np.max(np.abs(s2 - ref_shell)) < 1e-12 * np.abs(ref_shell).max()
    assert np.max(np.abs(t2 - ref_tilde)) < 1e-12 * np.abs(ref_shell).max()
