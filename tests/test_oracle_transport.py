"""Pins for the oracle's transport coupling (Sec. 6, velocities of Sec. 7)."""
import math

import numpy as np

from oracle import interp, lattice, transport as tr
from oracle.selfenergy import KB_EV
from paper_1604_03525_amd import inputs as I


def _sc(kg=(6, 6, 6)):
    m = I.toy_model(kg, kg)
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    return R, nd, lattice.grid_points(*kg)


def test_tight_binding_velocity_closed_form():
    """eps = -2 sum_a cos(k_a) on the simple-cubic lattice (a = 1, k Cartesian
    = 2 pi k_frac): v_a = 2 sin(2 pi k_frac,a)."""
    R, nd, _ = _sc()
    k = I.random_points(20, 5)
    v = tr.velocities(I.nn_hopping(R), R, nd, I.SC_VECTORS, k)
    want = 2.0 * np.sin(2 * np.pi * k)
    assert np.max(np.abs(v[:, 0, :] - want)) < 1e-12


def test_velocity_finite_differences_multiband():
    """Random 6-band fcc Hamiltonian: the analytic velocities equal central
    differences of the interpolated bands in Cartesian k (step 1e-5)."""
    R, nd = lattice.ws_vectors(I.FCC_METRIC, (3, 3, 3))
    HR = I.random_hamiltonian(R, I.FCC_VECTORS, 6, seed=7, scale=0.8)
    k = I.random_points(6, 8)
    v = tr.velocities(HR, R, nd, I.FCC_VECTORS, k)
    A = np.asarray(I.FCC_VECTORS)
    h = 1e-5
    for a in range(3):
        dk = np.zeros(3)
        dk[a] = h
        dfrac = A @ dk / (2 * np.pi)          # k_frac,i = a_i . k_cart / (2 pi)
        ep, _ = interp.bands(HR, R, nd, k + dfrac)
        em, _ = interp.bands(HR, R, nd, k - dfrac)
        fd = (ep - em) / (2 * h)
        assert np.max(np.abs(v[:, :, a] - fd)) < 1e-7 * np.abs(v).max()


def test_velocity_degenerate_copy():
    """Two identical decoupled bands: both carry the single band's velocity
    (the degenerate average of the velocity matrix diagonal)."""
    R, nd, _ = _sc()
    h = I.nn_hopping(R)[:, 0, 0]
    HR2 = h[:, None, None] * np.eye(2)[None]
    k = I.random_points(10, 6)
    v1 = tr.velocities(I.nn_hopping(R), R, nd, I.SC_VECTORS, k)
    v2 = tr.velocities(HR2, R, nd, I.SC_VECTORS, k)
    assert np.max(np.abs(v2 - v1[:, [0, 0], :])) < 1e-12


def test_lambda_tr_closed_form_einstein_constant_g():
    """Single band, Einstein modes, constant g: after the degenerate-mode
    average every mode has sum|c|^2 / (3 2 omega_E) and
      lambda_tr,q = that / (N(eps_F) omega_E) (1/N_k) sum_k d(eps_k - mu) d(eps_k+q - mu)
                    (1 - v_k . v_k+q / |v_k|^2)
    with the analytic band, velocity and Gaussian written out here (factor 1
    at the band extrema, where v = 0); at q = 0 only the extrema contribute."""
    R, nd, k = _sc((6, 6, 6))
    we = 0.05
    c = np.array([0.04, 0.01 - 0.02j, 0.03])
    HR, DR, gR = I.nn_hopping(R), I.einstein_dynmat(R, 3, we), I.constant_vertex(R, R, c)
    mu, sig = -1.0, 0.3
    q = np.vstack([np.zeros(3), k[[5, 17, 100]]])
    lam = tr.lambda_tr(HR, R, nd, DR, R, nd, gR, k, q, mu, sig, I.SC_VECTORS)

    def band(p):
        return -2.0 * sum(math.cos(2 * math.pi * x) for x in p)

    def vel(p):
        return np.array([2.0 * math.sin(2 * math.pi * x) for x in p])

    def delta(x):
        return math.exp(-(x / sig) ** 2) / (sig * math.sqrt(math.pi))

    dos = sum(delta(band(p) - mu) for p in k) / len(k)
    g2 = float(np.sum(np.abs(c) ** 2)) / (3 * 2 * we)
    scale = np.abs(lam).max()
    for iq, qq in enumerate(q):
        s = 0.0
        for p in k:
            vk, vq = vel(p), vel(p + qq)
            fac = 1.0 - float(vk @ vq) / float(vk @ vk) if float(vk @ vk) > 1e-18 else 1.0
            s += delta(band(p) - mu) * delta(band(p + qq) - mu) * fac
        want = g2 * s / len(k) / (dos * we)
        assert np.max(np.abs(lam[iq] - want)) < 1e-12 * scale
    assert np.all(lam[0] < 1e-2 * scale)


def test_eliashberg_function_weight_and_einstein():
    """int alpha^2 F d omega = (1/2) (1/N_q) sum omega lambda (the Gaussian has
    unit weight); a single Einstein frequency gives one Gaussian peak."""
    rng = np.random.default_rng(2)
    om = rng.uniform(0.01, 0.06, (40, 6))
    lam = rng.uniform(0.0, 2.0, (40, 6))
    w = np.linspace(-0.1, 0.2, 30001)
    a2f = tr.eliashberg_function(om, lam, w, 0.002)
    assert abs(np.trapezoid(a2f, w) - 0.5 * np.sum(om * lam) / 40) < 1e-10
    a2e = tr.eliashberg_function(np.full((5, 3), 0.03), np.full((5, 3), 0.7), w, 0.002)
    want = 0.5 * 3 * 0.03 * 0.7 * np.exp(-((w - 0.03) / 0.002) ** 2) / (0.002 * np.sqrt(np.pi))
    assert np.max(np.abs(a2e - want)) < 1e-12 * want.max()


def test_ziman_integral_einstein_and_high_temperature():
    """A narrow Einstein peak of weight A: rho n e^2/m_e -> 4 pi A omega_E n (1 + n)
    / (k_B T) (the peak width s adds a relative s^2 h''/(4 h) ~ 2e-5 for
    h = omega n (1 + n)); at high T, n (1 + n) -> (k_B T / omega)^2 and the
    integral grows linearly in T."""
    we, A, s = 0.03, 0.4, 1e-4
    w = np.linspace(0.0, 0.06, 60001)
    a2f = A * np.exp(-((w - we) / s) ** 2) / (s * np.sqrt(np.pi))
    for T in (100.0, 300.0):
        n = 1.0 / math.expm1(we / (KB_EV * T))
        want = 4 * np.pi * A * we * n * (1 + n) / (KB_EV * T)
        assert abs(tr.ziman_integral(w, a2f, T) / want - 1) < 1e-4
    r1 = tr.ziman_integral(w, a2f, 5000.0)
    r2 = tr.ziman_integral(w, a2f, 10000.0)
    assert abs(r2 / r1 - 2.0) < 1e-3
    assert tr.ziman_integral(w, a2f, 0.0) == 0.0
