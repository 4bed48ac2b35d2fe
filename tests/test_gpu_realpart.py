"""Real part of the electron self-energy on shell (Sec. 3 Eq. (3)) and its
Fermi-level-referenced form Sigma~' (Sec. 3 Eq. (5)): HIP path against the
FP64 oracle, through the C ABI.  Tolerances (infinity-norm relative error):
FP64 1e-10, FP32 1e-5, split-BF16 1e-4, as for Im Sigma."""
import sys

import numpy as np
import pytest

from oracle import realpart as rp
from paper_1604_03525_amd import epw
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


def _oracle(c, kidx=None):
    k = c["k"] if kidx is None else c["k"][kidx]
    return rp.resigma(c["HR"], c["R"], c["nd"], c["DR"], c["R"], c["nd"], c["gR"], k, c["q"],
                      c["T"], c["mu"], c["sigma"])


def _gpu(c, want_tilde=True, **kw):
    pts = epw.Points(c["k"], c["q"], c["kq"], device=DEV)
    shell, tilde = epw.epw_resigma(_system(c), pts, _params(c, **kw), want_tilde=want_tilde)
    return shell.cpu().numpy(), (None if tilde is None else tilde.cpu().numpy())


def _check(tag, got, ref, tol):
    for name, x, y in zip(("shell", "tilde"), got, ref):
        _say(tag, name, rel_err(x, y))
        assert np.abs(y).max() > 0
        assert rel_err(x, y) < tol


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "split_bf16"])
def test_toy_complete(dtype):
    """The 8^3 x 8^3 toy (single band, three modes), every k against every q."""
    c = toy_case()
    _check(("re toy", dtype), _gpu(c, dtype=dtype), _oracle(c), TOL[dtype])


@pytest.mark.parametrize("nb", [2, 5, 8, 16])
def test_fcc_band_counts(nb):
    """Band counts that pad to 2, 8, 8 and 16, FP64, whole and ragged q chunks
    (the chunks accumulate into both outputs)."""
    c = fcc_small_case(nb=nb, kg=(3, 3, 3), seed=nb)
    ref = _oracle(c)
    for chunk in (0, 7):
        _check(("re fcc nb", nb, "chunk", chunk), _gpu(c, chunk_q=chunk), ref, 1e-10)


def test_tilde_optional_and_shell_unchanged():
    """Skipping Sigma~' leaves Sigma' bit-identical."""
    c = fcc_small_case(nb=3, kg=(3, 3, 3), seed=2)
    a, t = _gpu(c)
    b, none = _gpu(c, want_tilde=False)
    assert none is None and t is not None
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "split_bf16"])
def test_offgrid_mobility_shape(dtype):
    """Random k and q with no k+q map (16 bands, 9 modes): the k+q states come
    from the per-pair interpolation and eigensolve."""
    c = mobility_small_case()
    _check(("re offgrid", dtype), _gpu(c, dtype=dtype), _oracle(c), TOL[dtype])


def test_realistic_full_size_sampled_k():
    """The benchmark workload (fcc, 8 bands, 6 modes, 279 WS, 20^3 k x 20^3 q)
    in the launch configuration of the benchmark, checked on sampled k points
    that the oracle evaluates one by one against all 8000 q."""
    c = realistic_case()
    got = _gpu(c)
    rng = np.random.default_rng(23)
    kidx = np.concatenate([[0, len(c["k"]) - 1], rng.choice(len(c["k"]), 3, replace=False)])
    ref = _oracle(c, kidx)
    _check("re realistic", (got[0][kidx], got[1][kidx]), ref, 1e-10)
