"""epw_imsigma_noalloc (Im Sigma with the library's static device scratch,
no allocation in the call) against epw_imsigma with a caller workspace:
bit-identical at the same q chunking, and to 1e-12 with the chunk the call
picks to fit its scratch; two calls in a row, the second smaller, so the
second runs on the first one's leftovers.  Sizes beyond the scratch are
rejected before any device work (checked on the CPU)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_1604_03525_amd import _lib, epw
from tests.helpers import fcc_small_case, mobility_small_case, rel_err, toy_case

DEV = "cuda"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _placeholder_structs(nk, nq, nb=16, nm=9, ne=617):
    # non-NULL placeholders: the size check rejects before any pointer is used
    keep = (ctypes.c_double * 4)()
    a = ctypes.cast(keep, ctypes.c_void_p)
    s = _lib.EpwSystem(nb, nm, ne, ne, a, a, a, a, a, a, a, 0, 0)
    p = _lib.EpwPoints(nk, nq, a, a, None, None, None)
    return s, p, a, keep


def test_noalloc_rejects_sizes_beyond_its_scratch():
    lib = _lib.load()
    # band tables alone exceed the scratch: 200,000 k x 16 x 16 complex128
    s, p, a, keep = _placeholder_structs(200000, 10)
    par = epw.make_params()
    assert lib.epw_imsigma_noalloc(ctypes.byref(s), ctypes.byref(p), ctypes.byref(par), a, None) \
        == _lib.EPW_ENOMEM
    assert b"one q point at a time" in lib.epw_last_error()
    # a given chunk that does not fit
    s, p, a, keep = _placeholder_structs(1000, 100000)
    par = epw.make_params(chunk_q=100000)
    assert lib.epw_imsigma_noalloc(ctypes.byref(s), ctypes.byref(p), ctypes.byref(par), a, None) \
        == _lib.EPW_ENOMEM
    assert b"chunk_q = 100000" in lib.epw_last_error()
    # argument errors come first, as in epw_imsigma
    par = epw.make_params(sigma=0.0)
    assert lib.epw_imsigma_noalloc(ctypes.byref(s), ctypes.byref(p), ctypes.byref(par), a, None) \
        == _lib.EPW_EINVAL


def _run_both(c, dtype, chunk_q):
    sysd = epw.System(c["R"], c["nd"], c["R"], c["nd"], c["HR"], c["DR"], c["gR"], DEV)
    pts = epw.Points(c["k"], c["q"], c["kq"], device=DEV)
    par = epw.make_params(T=c["T"], mu=c["mu"], sigma=c["sigma"], dtype=dtype, chunk_q=chunk_q)
    ref = epw.epw_imsigma(sysd, pts, par).cpu().numpy()
    got = epw.epw_imsigma_noalloc(sysd, pts, par).cpu().numpy()
    return got, ref


@pytest.mark.gpu
def test_noalloc_matches_workspace_call_two_calls():
    big = fcc_small_case(nb=3, kg=(4, 4, 4))
    small = toy_case((4, 4, 4))
    for name, c in (("fcc 3 bands 4^3 x 4^3", big), ("toy 4^3 x 4^3", small)):
        for dtype in ("fp64", "fp32"):
            _say("noalloc", name, dtype, "chunk_q 7")
            got, ref = _run_both(c, dtype, 7)
            assert np.abs(ref).max() > 0
            assert np.array_equal(got, ref), rel_err(got, ref)
            _say("noalloc", name, dtype, "auto chunk")
            got, ref = _run_both(c, dtype, 0)
            _say("  rel err", rel_err(got, ref))
            assert rel_err(got, ref) < 1e-12


@pytest.mark.gpu
def test_noalloc_offgrid_then_smaller():
    """Off-grid k+q (per-pair states in the scratch), then a smaller grid run."""
    c = mobility_small_case(nk=10, nq=13, nb=5, seed=35)
    _say("noalloc off-grid 5 bands 10 k x 13 q")
    got, ref = _run_both(c, "fp64", 4)
    assert np.array_equal(got, ref), rel_err(got, ref)
    got, ref = _run_both(c, "fp64", 0)
    assert rel_err(got, ref) < 1e-12
    s = toy_case((2, 2, 2))
    _say("noalloc toy 2^3")
    got, ref = _run_both(s, "fp64", 0)
    assert np.array_equal(got, ref) or rel_err(got, ref) < 1e-12
