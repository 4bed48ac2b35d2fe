"""epw_check_inputs: each failure code forced from the host with a bad input
built from a valid one (the valid inputs themselves pass)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from oracle import lattice
from paper_1604_03525_amd import _lib, epw
from tests.helpers import fcc_small_case, mobility_small_case

DEV = "cuda"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _code(c, herm_tol=1e-12, kq="grid", omega=None, evec=None, nmax=None):
    sysd = epw.System(c["R"], c["nd"], c["R"], c["nd"], c["HR"], c["DR"], c["gR"], DEV)
    if nmax is not None:
        sysd.nmax_e = nmax
    pts = epw.Points(c["k"], c["q"], c["kq"] if isinstance(kq, str) else kq, omega=omega, evec=evec, device=DEV)
    try:
        epw.epw_check_inputs(sysd, pts, herm_tol)
        return 0
    except epw.EpwError as e:
        _say("  ", e)
        return e.code


def test_check_inputs_arguments_on_host():
    """Argument errors are reported before any device work."""
    lib = _lib.load()
    keep = (ctypes.c_double * 4)()
    a = ctypes.cast(keep, ctypes.c_void_p)
    s = _lib.EpwSystem(3, 6, 19, 19, a, a, a, a, a, a, a, 0, 0)
    p = _lib.EpwPoints(8, 8, a, a, None, None, None)
    assert lib.epw_check_inputs(ctypes.byref(s), ctypes.byref(p), -1.0, a, 1 << 20, None) == _lib.EPW_EINVAL
    assert lib.epw_check_inputs(ctypes.byref(s), ctypes.byref(p), float("nan"), a, 1 << 20, None) == _lib.EPW_EINVAL
    assert lib.epw_check_inputs(ctypes.byref(s), ctypes.byref(p), 1e-12, None, 0, None) == _lib.EPW_ENOMEM
    par = epw.make_params()
    n = lib.epw_workspace_size(_lib.EPW_WS_CHECK, ctypes.byref(s), ctypes.byref(p), ctypes.byref(par))
    assert n > 0
    assert lib.epw_check_inputs(ctypes.byref(s), ctypes.byref(p), 1e-12, a, n - 1, None) == _lib.EPW_ENOMEM


@pytest.mark.gpu
def test_check_inputs_each_code():
    c = fcc_small_case(nb=3, kg=(4, 4, 4))
    _say("check: valid grid case")
    assert _code(c) == 0
    # 1. non-finite entries
    for key, val in (("HR", np.nan), ("gR", np.inf), ("DR", np.nan)):
        d = dict(c)
        d[key] = c[key].copy()
        d[key].reshape(-1)[7] = val
        _say("check: non-finite", key)
        assert _code(d) == _lib.EPW_EINVAL
    d = dict(c)
    d["k"] = c["k"].copy()
    d["k"][3, 1] = np.nan
    assert _code(d) == _lib.EPW_EINVAL
    # 2. degeneracy < 1, nmax_e below the largest component
    d = dict(c)
    d["nd"] = c["nd"].copy()
    d["nd"][5] = 0
    assert _code(d) == _lib.EPW_EINVAL
    m = mobility_small_case(nk=6, nq=7, nb=4)
    true_nmax = int(np.abs(m["R"]).max())
    assert true_nmax >= 2
    assert _code(m, kq=None, nmax=true_nmax) == 0
    assert _code(m, kq=None, nmax=true_nmax - 1) == _lib.EPW_EINVAL
    # 3. a WS set not closed under R -> -R
    d = dict(c)
    keep = np.ones(len(c["R"]), bool)
    keep[np.flatnonzero(np.any(c["R"] != 0, axis=1))[0]] = False
    d["R"], d["nd"] = c["R"][keep], c["nd"][keep]
    d["HR"], d["DR"], d["gR"] = c["HR"][keep], c["DR"][keep], c["gR"][keep][:, keep]
    _say("check: WS set without one negative")
    assert _code(d) == _lib.EPW_ESHAPE
    # 4. H(-R) != H(R)^dag, D(-R) != D(R)^T beyond the tolerance
    r = int(np.flatnonzero(np.any(c["R"] != 0, axis=1))[0])
    d = dict(c)
    d["HR"] = c["HR"].copy()
    d["HR"][r, 0, 1] += 1e-6
    _say("check: H(-R) != H(R)^dag")
    assert _code(d, herm_tol=1e-12) == _lib.EPW_ENOTHERM
    assert _code(d, herm_tol=1e-3) == 0
    d = dict(c)
    d["DR"] = c["DR"].copy()
    d["DR"][r, 0, 1] += 1e-9
    assert _code(d, herm_tol=1e-12) == _lib.EPW_ENOTHERM
    # 5. the k+q map: an entry out of range, a map that is not one-to-one
    kq = c["kq"].copy()
    kq[2, 3] = len(c["k"])
    assert _code(c, kq=kq) == _lib.EPW_EINVAL
    kq = c["kq"].copy()
    kq[2, 3] = kq[5, 3]
    _say("check: kq not one-to-one")
    assert _code(c, kq=kq) == _lib.EPW_EINVAL
    # given phonon states with a non-finite frequency
    om = np.full((len(c["q"]), 6), 0.02)
    ev = np.tile(np.eye(6, dtype=np.complex128), (len(c["q"]), 1, 1))
    assert _code(c, omega=om, evec=ev) == 0
    om[4, 2] = np.inf
    assert _code(c, omega=om, evec=ev) == _lib.EPW_EINVAL


@pytest.mark.gpu
def test_check_inputs_model_systems_pass():
    """The seeded model systems satisfy every check (off-grid: no map)."""
    c = mobility_small_case(nk=6, nq=7, nb=16)
    assert _code(c, kq=None) == 0
    m_R, m_nd = lattice.ws_vectors(np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]]), (6, 6, 6))
    assert len(m_R) == 279
