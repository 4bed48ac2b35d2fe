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


def test_spectral_workload_full_size_sampled():
    """The spectral-function workload of the benchmark (realistic fcc system,
    64 k on Gamma-X, 10^5 random q, 512 frequencies, FP64) in its launch
    configuration; the oracle evaluates two k points against all q at eight
    sampled frequencies and omega = 0, in q blocks."""
    c = realistic_case()
    wl = I.spectral_workload()
    c.update(k=wl["k"], q=wl["q"], kq=None)
    w = wl["wgrid"]
    A, sig, sig0, eps = _gpu(c, w, kq=False)
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
    _say("omega spectral workload sigma(w) %.2e sigma(0) %.2e A %.2e" % errs)
    assert max(errs) < 1e-10
    assert np.all(A >= 0) and np.all(np.isfinite(A))
