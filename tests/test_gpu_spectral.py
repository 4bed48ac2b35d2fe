"""Complex electron self-energy on a frequency grid (Sec. 3 Eq. (3)) and the
spectral function (Sec. 3 Eq. (10)): HIP path against the FP64 oracle,
through the C ABI.  Tolerances (infinity-norm relative error over the
compared block): FP64 1e-10, FP32 1e-5, split-BF16 1e-4, as for Im Sigma; the
spectral function, a rational function of Sigma, is compared with the same
bounds."""
import sys

import numpy as np
import pytest
import torch

from oracle import spectral as sp
from paper_1604_03525_amd import epw
from paper_1604_03525_amd import inputs as I
from tests.helpers import fcc_small_case, mobility_small_case, realistic_case, rel_err, toy_case

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = {"fp64": 1e-10, "fp32": 1e-5, "split_bf16": 1e-4}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _system(c):
    return epw.System(c["R"], c["nd"], c["R"], c["nd"], c["HR"], c["DR"], c["gR"], DEV)


def _params(c, **kw):
    base = dict(T=c["T"], mu=c["mu"], sigma=c["sigma"])
    base.update(kw)
    return epw.make_params(**base)


def _oracle(c, wgrid, kidx=None, q=None, nq_norm=None):
    k = c["k"] if kidx is None else c["k"][kidx]
    q = c["q"] if q is None else q
    return sp.selfenergy_omega(c["HR"], c["R"], c["nd"], c["DR"], c["R"], c["nd"], c["gR"], k, q,
                               c["T"], c["mu"], c["sigma"], wgrid, nq_norm=nq_norm)


def _gpu(c, wgrid, kq=True, **kw):
    pts = epw.Points(c["k"], c["q"], c["kq"] if kq else None, device=DEV)
    A, sig, sig0, eps = epw.spectral_function(_system(c), pts, _params(c, **kw), wgrid)
    return A.cpu().numpy(), sig.cpu().numpy(), sig0.cpu().numpy(), eps.cpu().numpy()


def _check(tag, got, ref, c, wgrid, tol):
    A, sig, sig0, _ = got
    rs, r0, reps = ref
    rA = sp.spectral_function(reps, c["mu"], wgrid, rs, r0)
    errs = (rel_err(sig, rs), rel_err(sig0, r0), rel_err(A, rA))
    _say(tag, "sigma(w) %.2e sigma(0) %.2e A %.2e" % errs)
    assert np.abs(rs).max() > 0 and np.all(A >= 0)
    assert max(errs) < tol


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "split_bf16"])
def test_toy_complete(dtype):
    """The 8^3 x 8^3 toy, every k against every q, 70 frequencies (two
    frequency tiles, the second ragged)."""
    c = toy_case()
    w = np.linspace(-1.5, 1.5, 70)
    _check(("omega toy", dtype), _gpu(c, w, dtype=dtype), _oracle(c, w), c, w, TOL[dtype])


@pytest.mark.parametrize("nb", [2, 5, 8, 16])
def test_fcc_band_counts(nb):
    """Band counts that pad to 2, 8, 8 and 16 (zero-padded records), FP64,
    whole and ragged q chunks (accumulated per chunk)."""
    c = fcc_small_case(nb=nb, kg=(3, 3, 3), seed=nb)
    w = np.linspace(-1.0, 1.0, 65)
    ref = _oracle(c, w)
    for chunk in (0, 7):
        _check(("omega fcc nb", nb, "chunk", chunk), _gpu(c, w, chunk_q=chunk), ref, c, w, 1e-10)


def test_no_frequencies_and_accumulate():
    """nw = 0 gives Sigma(0) alone; two q subsets with accumulate and
    nq_norm = N_q give the whole-set result."""
    c = fcc_small_case(nb=3, kg=(3, 3, 3), seed=2)
    sysd = _system(c)
    w = np.linspace(-0.7, 0.7, 9)
    full_s, full_0 = epw.epw_selfenergy_omega(sysd, epw.Points(c["k"], c["q"], None, device=DEV), _params(c), w)
    _, only0 = epw.epw_selfenergy_omega(sysd, epw.Points(c["k"], c["q"], None, device=DEV), _params(c),
                                        np.zeros(0))
    assert np.max(np.abs(only0.cpu().numpy() - full_0.cpu().numpy())) <= 1e-12 * np.abs(full_0.cpu().numpy()).max()
    nq = len(c["q"])
    s = torch.empty_like(full_s)
    s0 = torch.empty_like(full_0)
    for i, (a, b) in enumerate(((0, 11), (11, nq))):
        pts = epw.Points(c["k"], c["q"][a:b], None, device=DEV)
        epw.epw_selfenergy_omega(sysd, pts, _params(c, nq_norm=nq, accumulate=i > 0), w, out=s, out0=s0)
    ref, ref0, _ = _oracle(c, w)
    assert rel_err(s.cpu().numpy(), ref) < 1e-10
    assert rel_err(s0.cpu().numpy(), ref0) < 1e-10
    assert rel_err(full_s.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "split_bf16"])
def test_offgrid_mobility_shape(dtype):
    """Random k and q with no k+q map (16 bands, 9 modes): per-pair k+q
    states."""
    c = mobility_small_case()
    w = np.linspace(-0.5, 0.5, 40)
    _check(("omega offgrid", dtype), _gpu(c, w, kq=False, dtype=dtype), _oracle(c, w), c, w, TOL[dtype])


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "split_bf16"])
def test_k_outer_order(dtype):
    """The k-outer contraction order (R_e -> k once, R_p -> q per chunk, a
    per-pair rotation) on the toy, a 5-band fcc case with ragged chunks and
    the off-grid shape, against the same oracle."""
    cases = [("toy", toy_case(), True, np.linspace(-1.5, 1.5, 70)),
             ("fcc5", fcc_small_case(nb=5, kg=(3, 3, 3), seed=5), True, np.linspace(-1.0, 1.0, 65)),
             ("offgrid", mobility_small_case(), False, np.linspace(-0.5, 0.5, 40))]
    for name, c, kq, w in cases:
        ref = _oracle(c, w)
        for chunk in ((0, 7) if dtype == "fp64" else (0,)):
            _check(("omega k-outer", name, dtype, chunk), _gpu(c, w, kq=kq, dtype=dtype, chunk_q=chunk,
                                                                order="k_outer"), ref, c, w, TOL[dtype])


@pytest.mark.parametrize("order", ["k_inner", "k_outer"])
def test_polar_both_orders(order):
    """With the polar long-range term: the oracle's polar vertex summed with
    the frequency-resolved weights, both contraction orders."""
    from oracle import interp, lattice, polar
    from oracle.selfenergy import degenerate_average
    R, nd = lattice.ws_vectors(I.FCC_METRIC, (3, 3, 3))
    HR = I.random_hamiltonian(R, I.FCC_VECTORS, 4, seed=9, scale=0.8)
    DR = I.spring_dynmat(R, I.FCC_VECTORS, I.ATOMS_FCC2, shells=2, seed=10, scale=4e-4)
    gR = I.random_vertex(R, R, I.FCC_VECTORS, 6, 4, seed=11, g0=0.05)
    k = lattice.grid_points(3, 3, 3)
    par = I.polar_params()
    T, mu, d = 300.0, 0.1, 0.15
    w = np.linspace(-1.0, 1.0, 33)
    wall = np.concatenate([w, [0.0]])
    sig = np.zeros((len(k), 4, len(wall)), dtype=np.complex128)
    for ik, kk in enumerate(k):
        g, ek, ekq, om = polar.vertex_band(HR, R, nd, DR, R, nd, gR, kk, k, par)
        sig[ik] = sp.sigma_from_states(g, ekq, om, mu, T, d, wall, len(k))
    eps = interp.bands(HR, R, nd, k)[0]
    for iw in range(len(wall)):
        sig[:, :, iw] = (degenerate_average(eps, sig[:, :, iw].real, 1e-6)
                         + 1j * degenerate_average(eps, sig[:, :, iw].imag, 1e-6))
    sysd = epw.System(R, nd, R, nd, HR, DR, gR, DEV, polar=par)
    pts = epw.Points(k, k, lattice.kq_index((3, 3, 3), (3, 3, 3)), device=DEV)
    got, got0 = epw.epw_selfenergy_omega(sysd, pts, epw.make_params(T=T, mu=mu, sigma=d, order=order), w)
    e1, e0 = rel_err(got.cpu().numpy(), sig[:, :, :-1]), rel_err(got0.cpu().numpy(), sig[:, :, -1])
    _say("omega polar", order, e1, e0)
    assert max(e1, e0) < 1e-10


@pytest.mark.parametrize("order", ["auto", "k_inner"])
def test_spectral_workload_full_size_sampled(order):
    """The spectral-function workload of the benchmark (realistic fcc system,
    64 k on Gamma-X, 10^5 random q, 512 frequencies, FP64) in its launch
    configuration (auto: the k-outer order) and in the k-inner order; the
    oracle evaluates two k points against all q at eight sampled frequencies
    and omega = 0, in q blocks."""
    c = realistic_case()
    wl = I.spectral_workload()
    c.update(k=wl["k"], q=wl["q"], kq=None)
    w = wl["wgrid"]
    A, sig, sig0, eps = _gpu(c, w, kq=False, order=order)
    kidx = np.array([5, 40])
    jw = np.array([0, 77, 200, 255, 256, 300, 449, 511])
    nq = len(c["q"])
    rs = np.zeros((2, 8, len(jw)), dtype=np.complex128)
    r0 = np.zeros((2, 8), dtype=np.complex128)
    for a in range(0, nq, 25000):
        s_, s0_, reps = _oracle(c, w[jw], kidx, q=c["q"][a:a + 25000], nq_norm=nq)
        rs += s_
        r0 += s0_
    rA = sp.spectral_function(reps, c["mu"], w[jw], rs, r0)
    errs = (rel_err(sig[kidx][:, :, jw], rs), rel_err(sig0[kidx], r0), rel_err(A[kidx][:, :, jw], rA))
    _say("omega spectral workload", order, "sigma(w) %.2e sigma(0) %.2e A %.2e" % errs)
    assert max(errs) < 1e-10
    assert np.all(A >= 0) and np.all(np.isfinite(A))
