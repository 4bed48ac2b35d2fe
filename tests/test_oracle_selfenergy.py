"""Pins for the oracle's Im Sigma (Sec. 3 Eq. (8)) and reference gradient."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import interp, lattice, selfenergy as se, torch_ref
from paper_1604_03525_amd import inputs as I

KB = 8.617333262e-5


def _toy(kg=(8, 8, 8)):
    m = I.toy_model(kg, kg)
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    k = lattice.grid_points(*kg)
    return m, R, nd, k


def test_gaussian_normalisation_and_width():
    for s in (0.01, 0.05):
        area = integrate.quad(lambda x: se.gaussian(x, s), -np.inf, np.inf)[0]
        var = integrate.quad(lambda x: x * x * se.gaussian(x, s), -np.inf, np.inf)[0]
        assert abs(area - 1.0) < 1e-12
        assert abs(var - s * s / 2.0) < 1e-9 * s * s


def test_occupations_special_values():
    mu, T = 0.3, 250.0
    assert se.fermi(mu, mu, T) == 0.5
    x = np.linspace(-0.5, 0.5, 11)
    assert np.allclose(se.fermi(mu + x, mu, T) + se.fermi(mu - x, mu, T), 1.0, atol=1e-15)
    assert np.allclose(se.bose(x[x != 0], T) + se.bose(-x[x != 0], T), -1.0, atol=1e-12)
    w = 1e-6
    assert abs(se.bose(w, T) * w / (KB * T) - 1.0) < 1e-4          # n ~ kT/omega
    assert se.bose(0.1, 0.0) == 0.0
    assert list(se.fermi([-1.0, 0.0, 1.0], 0.0, 0.0)) == [1.0, 0.5, 0.0]
    assert se.fermi(100.0, 0.0, 1.0) == 0.0                             # no overflow NaN


def _closed_form(eps_k, eps_all, geff2, omega_e, mu, T, sigma):
    """pi g_eff^2 (1/N) sum_k' {[n + f'] d(e - e' + w) + [n + 1 - f'] d(e - e' - w)}
    with textbook n, f and the normalised Gaussian."""
    n = 0.0 if T == 0 else 1.0 / math.expm1(omega_e / (KB * T))
    out = np.zeros(len(eps_k))
    for i, e in enumerate(eps_k):
        s = 0.0
        for ep in eps_all:
            f = (1.0 if ep < mu else 0.0) if T == 0 else 1.0 / (math.exp((ep - mu) / (KB * T)) + 1.0)
            d1 = math.exp(-((e - ep + omega_e) / sigma) ** 2) / (sigma * math.sqrt(math.pi))
            d2 = math.exp(-((e - ep - omega_e) / sigma) ** 2) / (sigma * math.sqrt(math.pi))
            s += (n + f) * d1 + (n + 1.0 - f) * d2
        out[i] = math.pi * geff2 * s / len(eps_all)
    return out


def test_closed_form_einstein_constant_g():
    """P5: single band, Einstein phonons, constant g_a = c_a at R = 0:
    Im Sigma_k = pi (sum_a |c_a|^2 / 2 omega_E) (1/N) sum_k' {...} with the
    analytic band eps = -2 sum cos(2 pi k_a)."""
    m, R, nd, k = _toy((6, 6, 6))
    HR = I.nn_hopping(R)
    we = 0.06
    DR = I.einstein_dynmat(R, 3, we)
    c = np.array([0.05, 0.02j, -0.03 + 0.01j])
    gR = I.constant_vertex(R, R, c)
    ims = se.imsigma(HR, R, nd, DR, R, nd, gR, k, k, 300.0, 0.3, 0.08)
    eps = -2.0 * np.cos(2 * np.pi * k).sum(1)
    want = _closed_form(eps, eps, np.sum(np.abs(c) ** 2) / (2 * we), we, 0.3, 300.0, 0.08)
    assert np.max(np.abs(ims[:, 0] - want)) < 1e-12 * want.max()


def test_closed_form_dispersive_modes_single_axis():
    """P5b: toy phonons omega_a(q) = omega_max |sin pi q_a| with coupling to
    the x displacement only: Im Sigma_k = (pi/N) sum_q |c|^2/(2 omega_x(q))
    W(eps_k, eps_k+q, omega_x(q)), q_x = 0 plane cut.  Fails if the mode
    rotation uses rows instead of columns or the wrong frequency."""
    m, R, nd, k = _toy((6, 6, 6))
    HR, DR, _ = I.toy_arrays(R, R)
    c = 0.07
    gR = I.constant_vertex(R, R, [c, 0.0, 0.0])
    mu, T, sig = -0.2, 400.0, 0.1
    ims = se.imsigma(HR, R, nd, DR, R, nd, gR, k, k, T, mu, sig)
    eps = -2.0 * np.cos(2 * np.pi * k).sum(1)
    kq = lattice.kq_index((6, 6, 6), (6, 6, 6))
    want = np.zeros(len(k))
    for i in range(len(k)):
        s = 0.0
        for j in range(len(k)):
            w = 0.05 * abs(math.sin(math.pi * k[j, 0]))
            if w < 1e-3:
                continue
            n = 1.0 / math.expm1(w / (KB * T))
            ep = eps[kq[i, j]]
            f = 1.0 / (math.exp((ep - mu) / (KB * T)) + 1.0)
            g = lambda x: math.exp(-(x / sig) ** 2) / (sig * math.sqrt(math.pi))
            s += c * c / (2 * w) * ((n + f) * g(eps[i] - ep + w) + (n + 1 - f) * g(eps[i] - ep - w))
        want[i] = math.pi * s / len(k)
    assert np.max(np.abs(ims[:, 0] - want)) < 1e-12 * want.max()


def test_zero_temperature_dos_limit():
    """P5 at T -> 0 with mu far below the band: 2 Im Sigma = 1/tau =
    2 pi g_eff^2 D_sigma(eps_k - omega_E), the smeared density of states
    (Sec. 10.2 scattering rate; Im Sigma follows the DOS)."""
    m, R, nd, k = _toy((6, 6, 6))
    HR = I.nn_hopping(R)
    we = 0.05
    DR = I.einstein_dynmat(R, 3, we)
    c = np.array([0.04, 0.0, 0.03])
    gR = I.constant_vertex(R, R, c)
    sig = 0.3
    ims = se.imsigma(HR, R, nd, DR, R, nd, gR, k, k, 0.0, -100.0, sig)
    eps = -2.0 * np.cos(2 * np.pi * k).sum(1)
    geff2 = np.sum(np.abs(c) ** 2) / (2 * we)
    dos = np.array([np.mean(np.exp(-((e - we - eps) / sig) ** 2)) / (sig * math.sqrt(math.pi))
                    for e in eps])
    assert np.max(np.abs(2 * ims[:, 0] - 2 * math.pi * geff2 * dos)) < 1e-12 * dos.max()


def test_zero_temperature_blocking():
    """P9: at T = 0 with Einstein phonons, states within omega_E of mu cannot
    scatter; what remains is bounded by the Gaussian tail."""
    m, R, nd, k = _toy((8, 8, 8))
    HR = I.nn_hopping(R)
    we, sig = 0.5, 0.05
    DR = I.einstein_dynmat(R, 3, we)
    c = np.array([0.1, 0.1, 0.1])
    gR = I.constant_vertex(R, R, c)
    ims = se.imsigma(HR, R, nd, DR, R, nd, gR, k, k, 0.0, 0.0, sig)[:, 0]
    eps = -2.0 * np.cos(2 * np.pi * k).sum(1)
    geff2 = np.sum(np.abs(c) ** 2) / (2 * we)
    inside = np.abs(eps) < 0.25
    assert inside.sum() > 0
    bound = math.pi * geff2 * math.exp(-(0.25 / sig) ** 2) / (sig * math.sqrt(math.pi))
    assert np.all(ims[inside] <= bound)
    assert ims[~inside].max() > 1e6 * bound


def test_scaling_positivity_and_zero():
    """P8: Im Sigma(s g) = s^2 Im Sigma(g), Im Sigma(0) = 0, Im Sigma >= 0."""
    m, R, nd, k = _toy((4, 4, 4))
    HR, DR, gR = I.toy_arrays(R, R)
    a = se.imsigma(HR, R, nd, DR, R, nd, gR, k, k, m.T, m.mu, m.sigma)
    b = se.imsigma(HR, R, nd, DR, R, nd, 1.7 * gR, k, k, m.T, m.mu, m.sigma)
    z = se.imsigma(HR, R, nd, DR, R, nd, 0 * gR, k, k, m.T, m.mu, m.sigma)
    assert np.max(np.abs(b - 1.7 ** 2 * a)) < 1e-12 * a.max()
    assert np.all(z == 0)
    assert np.all(a >= 0)


def test_temperature_monotone_for_empty_band():
    """Raising T raises the rate (Sec. 10.2) when the band is empty."""
    m, R, nd, k = _toy((4, 4, 4))
    HR, DR, gR = I.toy_arrays(R, R)
    lo = se.imsigma(HR, R, nd, DR, R, nd, gR, k, k, 100.0, -50.0, m.sigma)
    hi = se.imsigma(HR, R, nd, DR, R, nd, gR, k, k, 400.0, -50.0, m.sigma)
    assert np.all(hi >= lo)


def test_gauge_invariance_degenerate_blocks():
    """P7: two identical decoupled bands (every k twofold degenerate) and
    Einstein phonons (threefold): random unitaries inside the degenerate
    blocks of U_k, U_k+q and e_q leave the averaged Im Sigma unchanged."""
    rng = np.random.default_rng(11)
    R, nd = lattice.ws_vectors(I.SC_METRIC, (3, 3, 3))
    k = lattice.grid_points(3, 3, 3)
    h = I.nn_hopping(R)[:, 0, 0]
    HR = h[:, None, None] * np.eye(2)[None]
    DR = I.einstein_dynmat(R, 3, 0.05)
    gR = I.random_vertex(R, R, I.SC_VECTORS, 3, 2, seed=3, g0=0.1)
    T, mu, sig = 300.0, 0.1, 0.2
    ref = se.imsigma(HR, R, nd, DR, R, nd, gR, k, k, T, mu, sig)

    def haar(n):
        z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        q, r = np.linalg.qr(z)
        return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]

    eps, U = interp.bands(HR, R, nd, k)
    om, e = interp.phonons(DR, R, nd, k)
    U2 = np.einsum("pij,pjk->pik", U, np.stack([haar(2) for _ in k]))
    e2 = np.einsum("pij,pjk->pik", e, np.stack([haar(3) for _ in k]))
    out = np.zeros((len(k), 2))
    raw_ref = np.zeros((len(k), 2))
    for ik, kk in enumerate(k):
        epq, Upq = interp.bands(HR, R, nd, kk[None] + k)
        Upq2 = np.einsum("pij,pjk->pik", Upq, np.stack([haar(2) for _ in k]))
        gw = interp.vertex_wannier(gR, R, nd, R, nd, kk, k)
        gb = interp.rotate(gw, U2[ik], Upq2, e2, om, 1e-3)
        out[ik] = se.imsigma_from_states(gb, eps[ik], epq, om, mu, T, sig, len(k))
        gb0 = interp.rotate(gw, U[ik], Upq, e, om, 1e-3)
        raw_ref[ik] = se.imsigma_from_states(gb0, eps[ik], epq, om, mu, T, sig, len(k))
    avg = se.degenerate_average(eps, out, 1e-6)
    assert np.max(np.abs(avg - ref)) < 1e-12 * ref.max()
    # the per-band values do depend on the gauge: the average is what is invariant
    assert np.max(np.abs(out - raw_ref)) > 1e-6 * ref.max()


def test_degenerate_average_groups():
    eps = np.array([[0.0, 1e-8, 0.5, 0.5 + 5e-7, 0.5 + 9e-7, 2.0]])
    v = np.array([[1.0, 3.0, 4.0, 5.0, 9.0, 7.0]])
    out = se.degenerate_average(eps, v, 1e-6)
    assert np.allclose(out, [[2.0, 2.0, 6.0, 6.0, 6.0, 7.0]])


def _realistic_small(kg=(3, 3, 3), nb=3, nm=6):
    R, nd = lattice.ws_vectors(I.FCC_METRIC, (2, 2, 2))
    HR = I.random_hamiltonian(R, I.FCC_VECTORS, nb, seed=1, scale=0.8)
    DR = I.spring_dynmat(R, I.FCC_VECTORS, I.ATOMS_FCC2, shells=2, seed=2, scale=4e-4)
    gR = I.random_vertex(R, R, I.FCC_VECTORS, nm, nb, seed=3, g0=0.05)
    k = lattice.grid_points(*kg)
    return R, nd, HR, DR, gR, k


def test_torch_reference_forward_matches_numpy_oracle():
    """The two independent forwards (different contraction orders, folded
    vs unfolded k+q) agree; toy model and a 3-band fcc model."""
    for case in ("toy", "fcc"):
        if case == "toy":
            m, R, nd, k = _toy((4, 4, 4))
            HR, DR, gR = I.toy_arrays(R, R)
            T, mu, sig, kg = m.T, m.mu, m.sigma, (4, 4, 4)
        else:
            R, nd, HR, DR, gR, k = _realistic_small()
            T, mu, sig, kg = 300.0, 0.1, 0.2, (3, 3, 3)
        om, e = interp.phonons(DR, R, nd, k)
        ref = se.imsigma(HR, R, nd, DR, R, nd, gR, k, k, T, mu, sig)
        kq = lattice.kq_index(kg, kg)
        w = I.loss_weights(len(k), HR.shape[1], 1)
        L, ims, *_ = torch_ref.loss_and_grads(gR, HR, om, e, w, Re=R, ndeg_e=nd, Rp=R, ndeg_p=nd,
                                              kpoints=k, qpoints=k, kq=kq, T=T, mu=mu, sigma=sig)
        assert np.max(np.abs(ims - ref)) < 1e-12 * ref.max()
        assert abs(L - np.sum(w * ref)) < 1e-12 * abs(L)


def test_reference_gradient_euler_and_finite_differences():
    """P10: L is homogeneous of degree 2 in g, so sum Re(conj(dL/dg) g) = 2L;
    the autograd gradients agree with central differences of the NumPy
    oracle's forward (h = 1e-6)."""
    R, nd, HR, DR, gR, k = _realistic_small((2, 2, 2), nb=2)
    T, mu, sig = 300.0, 0.1, 0.3
    om, e = interp.phonons(DR, R, nd, k)
    kq = lattice.kq_index((2, 2, 2), (2, 2, 2))
    w = I.loss_weights(len(k), 2, 1)
    kw = dict(Re=R, ndeg_e=nd, Rp=R, ndeg_p=nd, kpoints=k, qpoints=k, kq=kq, T=T, mu=mu, sigma=sig)
    L, ims, dg, dh, dom = torch_ref.loss_and_grads(gR, HR, om, e, w, **kw)
    assert abs(np.sum(np.real(np.conj(dg) * gR)) - 2 * L) < 1e-10 * abs(L)

    def loss(g=gR, h=HR, o=om):
        return np.sum(w * se.imsigma(h, R, nd, None, R, nd, g, k, k, T, mu, sig,
                                     phonon_states=(o, e)))
    rng = np.random.default_rng(4)
    hstep = 1e-6
    for _ in range(3):
        idx = tuple(rng.integers(0, s) for s in gR.shape)
        for unit in (1.0, 1j):
            gp = gR.copy(); gp[idx] += hstep * unit
            gm = gR.copy(); gm[idx] -= hstep * unit
            fd = (loss(g=gp) - loss(g=gm)) / (2 * hstep)
            an = dg[idx].real if unit == 1.0 else dg[idx].imag
            assert abs(fd - an) < 1e-6 * np.abs(dg).max()
        idx = tuple(rng.integers(0, s) for s in HR.shape)
        for unit in (1.0, 1j):
            hp = HR.copy(); hp[idx] += hstep * unit
            hm = HR.copy(); hm[idx] -= hstep * unit
            fd = (loss(h=hp) - loss(h=hm)) / (2 * hstep)
            an = dh[idx].real if unit == 1.0 else dh[idx].imag
            assert abs(fd - an) < 1e-6 * np.abs(dh).max()
        idx = (int(rng.integers(1, om.shape[0])), int(rng.integers(0, om.shape[1])))
        if om[idx] < 2e-3:
            continue
        op = om.copy(); op[idx] += hstep
        omm = om.copy(); omm[idx] -= hstep
        fd = (loss(o=op) - loss(o=omm)) / (2 * hstep)
        assert abs(fd - dom[idx]) < 1e-6 * np.abs(dom).max()


def test_reference_offgrid_forward_and_gradient():
    """The reference gradient's off-grid branch (no k+q map: H diagonalised at
    every unfolded k+q, as for the random point sets of Sec. 10.2) against the
    NumPy oracle: forward to 1e-12, Euler identity, and central differences
    (h = 1e-6) of the NumPy forward for dL/dg, dL/dH and dL/domega.  A wrong
    pairing of k+q states with (k, q) fails the forward check; a wrong
    Hermitisation or conjugation fails the dL/dH differences."""
    R, nd = lattice.ws_vectors(I.FCC_METRIC, (2, 2, 2))
    nb, nm = 3, 6
    HR = I.random_hamiltonian(R, I.FCC_VECTORS, nb, seed=41, scale=0.8)
    DR = I.spring_dynmat(R, I.FCC_VECTORS, I.ATOMS_FCC2, shells=2, seed=42, scale=4e-4)
    gR = I.random_vertex(R, R, I.FCC_VECTORS, nm, nb, seed=43, g0=0.05)
    k = I.random_points(4, 3)
    q = I.random_points(5, 2)
    T, mu, sig = 300.0, 0.1, 0.3
    om, e = interp.phonons(DR, R, nd, q)
    w = I.loss_weights(len(k), nb, 1)
    kw = dict(Re=R, ndeg_e=nd, Rp=R, ndeg_p=nd, kpoints=k, qpoints=q, kq=None, T=T, mu=mu, sigma=sig)
    L, ims, dg, dh, dom = torch_ref.loss_and_grads(gR, HR, om, e, w, **kw)

    def fwd(g=gR, h=HR, o=om):
        return se.imsigma(h, R, nd, None, R, nd, g, k, q, T, mu, sig, phonon_states=(o, e))

    ref = fwd()
    assert ref.max() > 0
    assert np.max(np.abs(ims - ref)) < 1e-12 * ref.max()
    # the k+q states really are per pair: pairing k with the k+q states of
    # another k changes the result far beyond the tolerance
    shuffled = se.imsigma(HR, R, nd, None, R, nd, gR, k, q, T, mu, sig, phonon_states=(om, e),
                          kq_points=(k[::-1][:, None, :] + q[None, :, :]))
    assert np.max(np.abs(shuffled - ref)) > 1e-3 * ref.max()
    assert abs(np.sum(np.real(np.conj(dg) * gR)) - 2 * L) < 1e-10 * abs(L)

    def loss(**a):
        return np.sum(w * fwd(**a))
    rng = np.random.default_rng(4)
    hstep = 1e-6
    for _ in range(3):
        idx = tuple(rng.integers(0, s) for s in gR.shape)
        for unit in (1.0, 1j):
            gp = gR.copy(); gp[idx] += hstep * unit
            gm = gR.copy(); gm[idx] -= hstep * unit
            fd = (loss(g=gp) - loss(g=gm)) / (2 * hstep)
            an = dg[idx].real if unit == 1.0 else dg[idx].imag
            assert abs(fd - an) < 1e-6 * np.abs(dg).max()
        for _h in range(2):
            idx = tuple(rng.integers(0, s) for s in HR.shape)
            for unit in (1.0, 1j):
                hp = HR.copy(); hp[idx] += hstep * unit
                hm = HR.copy(); hm[idx] -= hstep * unit
                fd = (loss(h=hp) - loss(h=hm)) / (2 * hstep)
                an = dh[idx].real if unit == 1.0 else dh[idx].imag
                assert abs(fd - an) < 1e-6 * np.abs(dh).max()
        idx = (int(rng.integers(0, om.shape[0])), int(rng.integers(0, om.shape[1])))
        if om[idx] < 2e-3:
            continue
        op = om.copy(); op[idx] += hstep
        omm = om.copy(); omm[idx] -= hstep
        fd = (loss(o=op) - loss(o=omm)) / (2 * hstep)
        assert abs(fd - dom[idx]) < 1e-6 * np.abs(dom).max()
