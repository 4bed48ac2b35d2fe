"""Pins for the oracle's phonon linewidth Pi''_q,nu (Sec. 3 Eq. (9)) and
coupling strength lambda_q,nu (Sec. 3 Eq. (11))."""
import itertools
import math

import numpy as np

from oracle import interp, lattice, phonon as ph
from paper_1604_03525_amd import inputs as I

KB = 8.617333262e-5


def _gauss(x, s):
    return math.exp(-(x / s) ** 2) / (s * math.sqrt(math.pi))


def _fd(e, mu, T):
    if T == 0.0:
        return 1.0 if e < mu else (0.0 if e > mu else 0.5)
    return 1.0 / (math.exp((e - mu) / (KB * T)) + 1.0)


def test_closed_form_einstein_constant_g():
    """Single band eps = -2 sum cos(2 pi k_a), Einstein phonons omega_E (three
    degenerate modes), constant g_a = c_a at R = 0.  Then |g_nu|^2 =
    |c_nu|^2 / (2 omega_E) and, after the average over the three degenerate
    modes,
      Pi''_q  = 2 pi (sum|c|^2 / 6 omega_E) / 3 (1/N) sum_k [f_k - f_k+q] d(e_k - e_k+q - omega_E)
      lambda_q = (sum|c|^2 / 6 omega_E) / (N(eF) omega_E) (1/N) sum_k d(e_k - mu) d(e_k+q - mu)
    (the second sum is the Gaussian nesting function of the band), written
    out with textbook loops over the grid and the analytic band."""
    # a hot, broad setting so that transitions between differently occupied
    # states (not Gaussian tails) dominate on this coarse grid
    kg = (8, 8, 8)
    m = I.toy_model(kg, kg)
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    k = lattice.grid_points(*kg)
    HR = I.nn_hopping(R)
    we = 0.15
    DR = I.einstein_dynmat(R, 3, we)
    c = np.array([0.05, 0.02j, -0.03 + 0.01j])
    gR = I.constant_vertex(R, R, c)
    T, mu, sig = 2000.0, 0.3, 0.25
    pi_im, lam = ph.phonon_selfenergy(HR, R, nd, DR, R, nd, gR, k, k, T, mu, sig)
    eps = -2.0 * np.cos(2 * np.pi * k).sum(1)
    kq = lattice.kq_index(kg, kg)
    N = len(k)
    g2 = float(np.sum(np.abs(c) ** 2)) / (2 * we) / 3.0
    dos = sum(_gauss(e - mu, sig) for e in eps) / N
    want_pi = np.zeros(N)
    want_lam = np.zeros(N)
    for j in range(N):
        sp = sl = 0.0
        for i in range(N):
            e, ep = eps[i], eps[kq[i, j]]
            sp += (_fd(e, mu, T) - _fd(ep, mu, T)) * _gauss(e - ep - we, sig)
            sl += _gauss(e - mu, sig) * _gauss(ep - mu, sig)
        want_pi[j] = 2 * math.pi * g2 * sp / N
        want_lam[j] = g2 * sl / N / (dos * we)
    for nu in range(3):
        assert np.max(np.abs(pi_im[:, nu] - want_pi)) < 1e-12 * np.abs(want_pi).max()
        assert np.max(np.abs(lam[:, nu] - want_lam)) < 1e-12 * want_lam.max()
    assert np.abs(want_pi).max() > 1e-6 and want_lam.max() > 1e-6      # not a test of tails


def _haar(rng, n):
    z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def test_brute_force_loops():
    """Every step written as explicit loops on a tiny system (2 bands, 3
    modes, SC coarse 2^3, 8 k x 8 q): vertex as the double Fourier sum,
    rotation by index loops, the Eq. (9) and Eq. (11) sums and the
    normalisations.  Agrees with the vectorised oracle to 1e-12."""
    R, nd = lattice.ws_vectors(I.SC_METRIC, (2, 2, 2))
    rng = np.random.default_rng(5)
    HR = I.random_hamiltonian(R, I.SC_VECTORS, 2, seed=7, decay=1.0, scale=0.5)
    DR = I.spring_dynmat(R, I.SC_VECTORS, I.ATOMS_SC1, shells=2, seed=8, scale=1e-3)
    gR = I.random_vertex(R, R, I.SC_VECTORS, 3, 2, seed=9, g0=0.1)
    k = lattice.grid_points(2, 2, 2)
    q = rng.random((8, 3))
    T, mu, sig = 500.0, 0.0, 0.2
    pi_im, lam = ph.phonon_selfenergy(HR, R, nd, DR, R, nd, gR, k, q, T, mu, sig, deg_tol=0.0)

    def herm_eigh(X):
        return np.linalg.eigh(0.5 * (X + X.conj().T))

    def interp1(XR, p):
        out = np.zeros(XR.shape[1:], dtype=np.complex128)
        for r in range(len(R)):
            out += np.exp(2j * np.pi * np.dot(p, R[r])) * XR[r] / nd[r]
        return out

    P = np.zeros((len(q), 3))
    L = np.zeros((len(q), 3))
    eks = []
    for kk in k:
        ek, Uk = herm_eigh(interp1(HR, kk))
        eks.append(ek)
        for iq, qq in enumerate(q):
            lam_ph, e = np.linalg.eigh(0.5 * (interp1(DR.astype(np.complex128), qq) +
                                              interp1(DR.astype(np.complex128), qq).conj().T))
            w = np.sign(lam_ph) * np.sqrt(np.abs(lam_ph))
            ekq, Ukq = herm_eigh(interp1(HR, kk + qq))
            gw = np.zeros((3, 2, 2), dtype=np.complex128)
            for a, b in itertools.product(range(len(R)), range(len(R))):
                gw += np.exp(2j * np.pi * (np.dot(kk, R[a]) + np.dot(qq, R[b]))) * gR[a, b] / (nd[a] * nd[b])
            for nu in range(3):
                if w[nu] < 1e-3:
                    continue
                for mm, nn in itertools.product(range(2), range(2)):
                    g = 0.0j
                    for al, i, j in itertools.product(range(3), range(2), range(2)):
                        g += np.conj(Ukq[i, mm]) * gw[al, i, j] * e[al, nu] * Uk[j, nn]
                    g2 = abs(g) ** 2 / (2 * w[nu])
                    P[iq, nu] += g2 * (_fd(ek[nn], mu, T) - _fd(ekq[mm], mu, T)) * _gauss(ek[nn] - ekq[mm] - w[nu], sig)
                    L[iq, nu] += g2 * _gauss(ek[nn] - mu, sig) * _gauss(ekq[mm] - mu, sig)
    N = len(k)
    dos = sum(_gauss(x - mu, sig) for e in eks for x in e) / N
    om, _ = interp.phonons(DR, R, nd, q)
    want_pi = 2 * math.pi * P / N
    want_lam = np.where(om >= 1e-3, L / (N * dos * np.where(om >= 1e-3, om, 1.0)), 0.0)
    assert np.max(np.abs(pi_im - want_pi)) < 1e-12 * np.abs(want_pi).max()
    assert np.max(np.abs(lam - want_lam)) < 1e-12 * np.abs(want_lam).max()


def test_scaling_and_zero_coupling():
    """Pi'' and lambda are quadratic in g and vanish with it."""
    m = I.toy_model((4, 4, 4), (4, 4, 4))
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    k = lattice.grid_points(4, 4, 4)
    HR, DR, gR = I.toy_arrays(R, R)
    a = ph.phonon_selfenergy(HR, R, nd, DR, R, nd, gR, k, k, 300.0, -0.5, 0.1)
    b = ph.phonon_selfenergy(HR, R, nd, DR, R, nd, 1.7 * gR, k, k, 300.0, -0.5, 0.1)
    z = ph.phonon_selfenergy(HR, R, nd, DR, R, nd, 0.0 * gR, k, k, 300.0, -0.5, 0.1)
    for x, y, zz in zip(a, b, z):
        assert np.max(np.abs(y - 1.7 ** 2 * x)) < 1e-12 * np.abs(y).max()
        assert np.all(zz == 0.0)


def test_zero_temperature_empty_band():
    """T = 0 with mu far below the band: every f is 0, so Pi'' = 0 exactly."""
    m = I.toy_model((4, 4, 4), (4, 4, 4))
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    k = lattice.grid_points(4, 4, 4)
    HR, DR, gR = I.toy_arrays(R, R)
    pi_im, lam = ph.phonon_selfenergy(HR, R, nd, DR, R, nd, gR, k, k, 0.0, -20.0, 0.1)
    assert np.all(pi_im == 0.0)
    assert np.max(lam) < 1e-300 or np.all(lam == 0.0)


def test_gauge_invariance_degenerate_modes_and_bands():
    """Two identical decoupled bands and Einstein phonons: random unitaries
    inside the degenerate blocks of U_k, U_k+q and e_q leave the mode-averaged
    Pi'' and lambda unchanged, while the per-mode values do change."""
    rng = np.random.default_rng(12)
    R, nd = lattice.ws_vectors(I.SC_METRIC, (3, 3, 3))
    k = lattice.grid_points(3, 3, 3)
    h = I.nn_hopping(R)[:, 0, 0]
    HR = h[:, None, None] * np.eye(2)[None]
    DR = I.einstein_dynmat(R, 3, 0.05)
    gR = I.random_vertex(R, R, I.SC_VECTORS, 3, 2, seed=3, g0=0.1)
    T, mu, sig = 300.0, 0.1, 0.2
    ref_pi, ref_lam = ph.phonon_selfenergy(HR, R, nd, DR, R, nd, gR, k, k, T, mu, sig)
    eps, U = interp.bands(HR, R, nd, k)
    om, e = interp.phonons(DR, R, nd, k)
    U2 = np.einsum("pij,pjk->pik", U, np.stack([_haar(rng, 2) for _ in k]))
    e2 = np.einsum("pij,pjk->pik", e, np.stack([_haar(rng, 3) for _ in k]))
    P = np.zeros(om.shape)
    P0 = np.zeros(om.shape)
    L = np.zeros(om.shape)
    for ik, kk in enumerate(k):
        epq, Upq = interp.bands(HR, R, nd, kk[None] + k)
        Upq2 = np.einsum("pij,pjk->pik", Upq, np.stack([_haar(rng, 2) for _ in k]))
        gw = interp.vertex_wannier(gR, R, nd, R, nd, kk, k)
        p, l = ph.phonon_sums_one_k(interp.rotate(gw, U2[ik], Upq2, e2, om, 1e-3), eps[ik], epq, om, mu, T, sig)
        p0, _ = ph.phonon_sums_one_k(interp.rotate(gw, U[ik], Upq, e, om, 1e-3), eps[ik], epq, om, mu, T, sig)
        P += p
        P0 += p0
        L += l
    N = len(k)
    from oracle.selfenergy import degenerate_average
    pi2 = degenerate_average(om, 2 * np.pi * P / N, 1e-6)
    lam2 = degenerate_average(om, L / (N * ph.dos_at_fermi(eps, mu, sig) * om), 1e-6)
    assert np.max(np.abs(pi2 - ref_pi)) < 1e-12 * np.abs(ref_pi).max()
    assert np.max(np.abs(lam2 - ref_lam)) < 1e-12 * np.abs(ref_lam).max()
    assert np.max(np.abs(P - P0)) > 1e-6 * np.abs(P0).max()


def test_q_outer_order_matches_k_outer_order():
    """The q-outer evaluation (R_p first, all k at once) equals the k-outer
    one: a different order of the same finite sums (fcc, 3 bands)."""
    R, nd = lattice.ws_vectors(I.FCC_METRIC, (2, 2, 2))
    HR = I.random_hamiltonian(R, I.FCC_VECTORS, 3, seed=4, decay=1.5, scale=0.8)
    DR = I.spring_dynmat(R, I.FCC_VECTORS, I.ATOMS_FCC2, shells=2, seed=5, scale=2e-3)
    gR = I.random_vertex(R, R, I.FCC_VECTORS, 6, 3, seed=6, g0=0.05)
    k = lattice.grid_points(3, 3, 3)
    q = np.random.default_rng(8).random((5, 3))
    a = ph.phonon_selfenergy(HR, R, nd, DR, R, nd, gR, k, q, 600.0, 0.2, 0.15)
    b = ph.phonon_selfenergy(HR, R, nd, DR, R, nd, gR, k, q, 600.0, 0.2, 0.15, loop="q")
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) < 1e-12 * np.abs(x).max()
