"""Pins for the oracle's complex electron self-energy on a frequency grid
(Sec. 3 Eq. (3)), Sigma~' (Sec. 3 Eq. (5)) and the spectral function
(Sec. 3 Eq. (10))."""
import math

import numpy as np

from oracle import interp, lattice, realpart as rp, spectral as sp
from oracle.selfenergy import degenerate_average
from paper_1604_03525_amd import inputs as I

KB = 8.617333262e-5


def _toy(kg):
    m = I.toy_model(kg, kg)
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    return R, nd, lattice.grid_points(*kg)


def _fd(e, mu, T):
    return 1.0 / (math.exp((e - mu) / (KB * T)) + 1.0)


def _einstein(kg=(5, 5, 5), we=0.06, c=(0.05, 0.02j, -0.03 + 0.01j)):
    R, nd, k = _toy(kg)
    HR = I.nn_hopping(R)
    DR = I.einstein_dynmat(R, 3, we)
    gR = I.constant_vertex(R, R, np.array(c))
    return R, nd, k, HR, DR, gR


def test_closed_form_einstein_constant_g():
    """Single band eps = -2 sum cos(2 pi k_a), Einstein phonons, constant g
    (sum_nu |g_nu|^2 = sum|c|^2 / (2 omega_E)): Sigma_k(omega) is the mean over
    k' of the two complex poles, written with Python complex arithmetic on the
    analytic band; the same at omega = 0."""
    c = np.array([0.05, 0.02j, -0.03 + 0.01j])
    we = 0.06
    R, nd, k, HR, DR, gR = _einstein(we=we, c=c)
    T, mu, d = 300.0, 0.3, 0.05
    wgrid = np.linspace(-1.0, 1.0, 9)
    kk = k[[0, 7, 31]]
    sig, sig0, eps_k = sp.selfenergy_omega(HR, R, nd, DR, R, nd, gR, kk, k, T, mu, d, wgrid)
    eps = -2.0 * np.cos(2 * np.pi * k).sum(1)
    g2 = float(np.sum(np.abs(c) ** 2)) / (2 * we)
    n = 1.0 / math.expm1(we / (KB * T))

    def s(w):
        acc = 0j
        for ep in eps:
            f = _fd(ep, mu, T)
            acc += (n + f) / complex(w - (ep - mu) + we, d) + (n + 1 - f) / complex(w - (ep - mu) - we, d)
        return g2 * acc / len(eps)

    want = np.array([s(w) for w in wgrid])
    scale = np.abs(want).max()
    for i in range(3):
        assert np.max(np.abs(sig[i, 0] - want)) < 1e-12 * scale
        assert abs(sig0[i, 0] - s(0.0)) < 1e-12 * scale
    # a single band with constant g: Sigma does not depend on k
    assert np.allclose(eps_k[:, 0], -2.0 * np.cos(2 * np.pi * kk).sum(1), atol=1e-12)


def test_retarded_sign_and_high_frequency_tail():
    """Every pole weight n + f and n + 1 - f is >= 0 and the poles sit below
    the real axis, so Im Sigma <= 0 at every omega; far from all poles
    omega Sigma(omega) -> (1/N_q) sum |g|^2 (2 n_q,nu + 1), which for constant
    g is sum|c|^2 (2 n + 1) / (2 omega_E)."""
    c = np.array([0.04, -0.01 + 0.03j, 0.02])
    we = 0.05
    R, nd, k, HR, DR, gR = _einstein(kg=(4, 4, 4), we=we, c=c)
    T = 500.0
    wgrid = np.concatenate([np.linspace(-8.0, 8.0, 41), [1e7]])
    sig, _, _ = sp.selfenergy_omega(HR, R, nd, DR, R, nd, gR, k[:3], k, T, 0.2, 0.03, wgrid)
    assert np.all(sig[:, :, :-1].imag <= 0.0)
    n = 1.0 / math.expm1(we / (KB * T))
    total = float(np.sum(np.abs(c) ** 2)) * (2 * n + 1) / (2 * we)
    assert np.max(np.abs(1e7 * sig[:, 0, -1] - total)) < 1e-6 * total


def _whole_line(n, s=1.0):
    """Nodes omega = s tan t on an even grid in t over (-pi/2, pi/2) and the
    trapezoid weights of d omega = s sec^2 t dt: integrals over the whole
    real line of functions decaying like 1/omega^2."""
    t = np.linspace(-np.pi / 2, np.pi / 2, n + 2)[1:-1]
    return s * np.tan(t), s * (t[1] - t[0]) / np.cos(t) ** 2


def test_lorentzian_weight_sum_rule():
    """-(1/pi) integral Im Sigma(omega) d omega over the real line = the total
    pole weight (1/N_q) sum |g|^2 (2 n + 1): each pole's imaginary part is a
    unit-area Lorentzian of width delta.  The integrand times sec^2 t tends
    to delta x weight at t = +-pi/2, so the two end nodes left out of the
    trapezoid hold about delta (t_1 - t_0) of the weight (~3e-6 here)."""
    c = np.array([0.03, 0.02, 0.01j])
    we = 0.07
    R, nd, k, HR, DR, gR = _einstein(kg=(3, 3, 3), we=we, c=c)
    T, d = 300.0, 0.05
    w, dw = _whole_line(60001)
    sig, _, _ = sp.selfenergy_omega(HR, R, nd, DR, R, nd, gR, k[:1], k, T, 0.0, d, w)
    area = -np.sum(sig[0, 0].imag * dw) / np.pi
    n = 1.0 / math.expm1(we / (KB * T))
    total = float(np.sum(np.abs(c) ** 2)) * (2 * n + 1) / (2 * we)
    assert abs(area - total) < 5e-6 * total


def test_real_part_matches_on_shell_oracle():
    """At omega = eps_nk - mu the real part is Sigma' of the on-shell module
    (real x / (x^2 + delta^2) weights), and Re Sigma(0) is Sigma' - Sigma~'."""
    R, nd, k = _toy((4, 4, 4))
    HR, DR, gR = I.toy_arrays(R, R)
    T, mu, d = 300.0, -0.5, 0.08
    shell, tilde = rp.resigma(HR, R, nd, DR, R, nd, gR, k[:4], k, T, mu, d)
    for i in range(4):
        e = interp.bands(HR, R, nd, k[i:i + 1])[0][0, 0]
        sig, sig0, _ = sp.selfenergy_omega(HR, R, nd, DR, R, nd, gR, k[i:i + 1], k, T, mu, d, [e - mu])
        assert abs(sig[0, 0, 0].real - shell[i, 0]) < 1e-12 * abs(shell).max()
        assert abs(sig0[0, 0].real - (shell[i, 0] - tilde[i, 0])) < 1e-12 * abs(shell).max()


def test_scaling_and_gauge_invariance():
    """Sigma(omega) is quadratic in g; with two identical decoupled bands,
    random unitaries in the degenerate blocks of U_k, U_k+q and e_q leave the
    band-averaged Sigma(omega) unchanged."""
    rng = np.random.default_rng(5)
    R, nd = lattice.ws_vectors(I.SC_METRIC, (3, 3, 3))
    k = lattice.grid_points(3, 3, 3)
    h = I.nn_hopping(R)[:, 0, 0]
    HR = h[:, None, None] * np.eye(2)[None]
    DR = I.einstein_dynmat(R, 3, 0.05)
    gR = I.random_vertex(R, R, I.SC_VECTORS, 3, 2, seed=4, g0=0.1)
    T, mu, d = 300.0, 0.1, 0.1
    wgrid = np.linspace(-0.6, 0.6, 7)
    ref, ref0, eps = sp.selfenergy_omega(HR, R, nd, DR, R, nd, gR, k, k, T, mu, d, wgrid)
    big, _, _ = sp.selfenergy_omega(HR, R, nd, DR, R, nd, 1.7 * gR, k, k, T, mu, d, wgrid)
    assert np.max(np.abs(big - 1.7 ** 2 * ref)) < 1e-12 * np.abs(big).max()

    def haar(n):
        z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        q, r = np.linalg.qr(z)
        return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]

    eps_k, U = interp.bands(HR, R, nd, k)
    om, e = interp.phonons(DR, R, nd, k)
    U2 = np.einsum("pij,pjk->pik", U, np.stack([haar(2) for _ in k]))
    e2 = np.einsum("pij,pjk->pik", e, np.stack([haar(3) for _ in k]))
    raw = np.zeros((len(k), 2, len(wgrid)), dtype=np.complex128)
    for ik, kk in enumerate(k):
        epq, Upq = interp.bands(HR, R, nd, kk[None] + k)
        Upq2 = np.einsum("pij,pjk->pik", Upq, np.stack([haar(2) for _ in k]))
        gw = interp.vertex_wannier(gR, R, nd, R, nd, kk, k)
        raw[ik] = sp.sigma_from_states(interp.rotate(gw, U2[ik], Upq2, e2, om, 1e-3), epq, om, mu, T, d,
                                       wgrid, len(k))
    for iw in range(len(wgrid)):
        got = (degenerate_average(eps_k, raw[:, :, iw].real, 1e-6)
               + 1j * degenerate_average(eps_k, raw[:, :, iw].imag, 1e-6))
        assert np.max(np.abs(got - ref[:, :, iw])) < 1e-12 * np.abs(ref).max()


def test_spectral_function_constant_self_energy_peak_and_width():
    """With Sigma(omega) = a - i G at every omega and Re Sigma(0) = b, A is a
    peak at the solution of the Dyson condition omega = xi + (a - b) whose full
    width at half maximum is 2 G (the squared Sigma'' of the denominator; the
    unsquared form would give 2 sqrt(G)), found on a fine grid."""
    xi, a, b, G = 0.13, 0.05, 0.02, 0.004
    w = np.linspace(-0.5, 0.5, 200001)
    sig = np.full((1, 1, len(w)), a - 1j * G)
    A = sp.spectral_function(np.array([[xi + 0.4]]), 0.4, w, sig, np.array([[b + 0.3j]]))[0, 0]
    i = int(np.argmax(A))
    assert abs(w[i] - (xi + a - b)) < 1e-5
    half = A >= A[i] / 2
    width = w[half][-1] - w[half][0]
    assert abs(width - 2 * G) < 2e-5
    assert abs(A[i] - 1.0 / (np.pi * G)) < 1e-6 / G


def test_spectral_function_sum_rule_interacting():
    """A_nk = -(1/pi) Im G with G = 1/(omega - xi - Sigma(omega) + Re Sigma(0))
    and Sigma a finite sum of retarded poles: integral A d omega = 1 over the
    real line."""
    R, nd, k = _toy((4, 4, 4))
    HR, DR, gR = I.toy_arrays(R, R)
    w, dw = _whole_line(60001)
    sig, sig0, eps = sp.selfenergy_omega(HR, R, nd, DR, R, nd, gR, k[:2], k, 300.0, -0.5, 0.05, w)
    A = sp.spectral_function(eps, -0.5, w, sig, sig0)
    assert np.all(A >= 0)
    for i in range(2):
        assert abs(np.sum(A[i, 0] * dw) - 1.0) < 1e-9
