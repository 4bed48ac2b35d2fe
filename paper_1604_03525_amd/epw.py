"""Python binding of libepw with the same call names as include/epw.h.

Argument marshalling only: host integer steps take and return NumPy arrays;
device steps take torch tensors on a HIP device (torch provides the memory
and the current stream) and every arithmetic step runs in libepw's kernels.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (EPW_FP32, EPW_FP64, EPW_SPLIT_BF16, EPW_WS_CHECK, EPW_WS_IMSIGMA,  # noqa: F401
                   EPW_WS_IMSIGMA_BACKWARD, EPW_WS_INTERP_G, EPW_WS_PHONON, EPW_WS_RESIGMA,
                   EPW_WS_TRANSPORT, EpwError)

DTYPES = {"fp64": EPW_FP64, "fp32": EPW_FP32, "split_bf16": EPW_SPLIT_BF16}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(t, dtype, device):
    """Contiguous device tensor of the given dtype (no copy when already so)."""
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    return t.to(device=device, dtype=dtype).contiguous()


# ------------------------------------------------------------------ host steps

def epw_ws_vectors(metric, ncell):
    """Wigner-Seitz vectors and degeneracies (host, exact)."""
    lib = _lib.load()
    m = np.ascontiguousarray(np.asarray(metric, dtype=np.int64).reshape(9))
    n = np.ascontiguousarray(np.asarray(ncell, dtype=np.int32).reshape(3))
    count = ctypes.c_int32(0)
    i32p = ctypes.POINTER(ctypes.c_int32)
    rc = lib.epw_ws_vectors(m.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n.ctypes.data_as(i32p),
                            None, None, 0, ctypes.byref(count))
    if rc not in (_lib.EPW_OK, _lib.EPW_ENOMEM):
        _lib.check(rc)
    R = np.zeros((count.value, 3), dtype=np.int32)
    nd = np.zeros(count.value, dtype=np.int32)
    _lib.check(lib.epw_ws_vectors(m.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n.ctypes.data_as(i32p),
                                  R.ctypes.data_as(i32p), nd.ctypes.data_as(i32p), count.value,
                                  ctypes.byref(count)))
    return R, nd


def epw_grid_points(n):
    lib = _lib.load()
    nn = np.ascontiguousarray(np.asarray(n, dtype=np.int32).reshape(3))
    out = np.zeros((int(np.prod(nn)), 3), dtype=np.float64)
    _lib.check(lib.epw_grid_points(nn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def epw_kq_index(kgrid, qgrid):
    lib = _lib.load()
    kg = np.ascontiguousarray(np.asarray(kgrid, dtype=np.int32).reshape(3))
    qg = np.ascontiguousarray(np.asarray(qgrid, dtype=np.int32).reshape(3))
    out = np.zeros((int(np.prod(kg)), int(np.prod(qg))), dtype=np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    _lib.check(lib.epw_kq_index(kg.ctypes.data_as(i32p), qg.ctypes.data_as(i32p), out.ctypes.data_as(i32p)))
    return out


# ---------------------------------------------------------------- device steps

def epw_interp_bands(HR, R, ndeg, kfrac):
    """(eps [nk][nb] float64, U [nk][nb][nb] complex128) on the device of HR."""
    lib = _lib.load()
    dev = HR.device
    HR = _dev(HR, torch.complex128, dev)
    R = _dev(R, torch.int32, dev)
    ndeg = _dev(ndeg, torch.int32, dev)
    k = _dev(kfrac, torch.float64, dev)
    nb, nk = HR.shape[-1], k.shape[0]
    eps = torch.empty((nk, nb), dtype=torch.float64, device=dev)
    U = torch.empty((nk, nb, nb), dtype=torch.complex128, device=dev)
    _lib.check(lib.epw_interp_bands(nb, R.shape[0], _ptr(R), _ptr(ndeg), _ptr(HR), nk, _ptr(k),
                                    _ptr(eps), _ptr(U), _stream(dev)))
    return eps, U


def epw_interp_phonons(DR, R, ndeg, qfrac):
    """(omega [nq][nm] float64, evec [nq][nm][nm] complex128)."""
    lib = _lib.load()
    dev = DR.device
    DR = _dev(DR, torch.float64, dev)
    R = _dev(R, torch.int32, dev)
    ndeg = _dev(ndeg, torch.int32, dev)
    q = _dev(qfrac, torch.float64, dev)
    nm, nq = DR.shape[-1], q.shape[0]
    om = torch.empty((nq, nm), dtype=torch.float64, device=dev)
    ev = torch.empty((nq, nm, nm), dtype=torch.complex128, device=dev)
    _lib.check(lib.epw_interp_phonons(nm, R.shape[0], _ptr(R), _ptr(ndeg), _ptr(DR), nq, _ptr(q),
                                      _ptr(om), _ptr(ev), _stream(dev)))
    return om, ev


class System:
    """Device-resident real-space system: WS sets, H(R_e), D(R_p), g(R_e,R_p)."""

    def __init__(self, Re, ndeg_e, Rp, ndeg_p, HR, DR, gR, device="cuda", polar=None):
        self.device = torch.device(device)
        self.polar = None if polar is None else make_polar(**polar)
        d = self.device
        self.Re = _dev(Re, torch.int32, d)
        self.ndeg_e = _dev(ndeg_e, torch.int32, d)
        self.Rp = _dev(Rp, torch.int32, d)
        self.ndeg_p = _dev(ndeg_p, torch.int32, d)
        self.HR = _dev(HR, torch.complex128, d)
        self.DR = None if DR is None else _dev(DR, torch.float64, d)
        self.gR = _dev(gR, torch.complex128, d)
        self.nb = self.HR.shape[-1]
        self.nm = self.gR.shape[2]
        # largest |R_e| component: lets the kernels generate the electron phases
        Rh = np.asarray(Re.cpu() if isinstance(Re, torch.Tensor) else Re)
        nmax = int(np.abs(Rh).max()) if Rh.size else 0
        self.nmax_e = nmax if 1 <= nmax <= _lib.EPW_MAX_NMAX else 0

    def c_struct(self):
        s = _lib.EpwSystem(self.nb, self.nm, self.Re.shape[0], self.Rp.shape[0],
                           _ptr(self.Re), _ptr(self.ndeg_e), _ptr(self.Rp), _ptr(self.ndeg_p),
                           _ptr(self.HR), _ptr(self.DR), _ptr(self.gR), self.nmax_e, 0)
        if self.polar is not None:
            s.polar = ctypes.cast(ctypes.pointer(self.polar), ctypes.c_void_p)
        return s


def make_polar(vectors, tau, zstar, eps_inf, masses, prefactor, alpha, cutoff):
    """The long-range (polar) data of Sec. 4 as the host struct of the C ABI:
    primitive vectors [3][3] (rows), positions tau [nat][3], Born charges
    zstar [nat][3][3], eps_inf [3][3], masses [nat] (Cartesian, one length
    unit), the overall factor C, the Gaussian parameter and the cutoff."""
    tau = np.asarray(tau, dtype=np.float64)
    nat = len(tau)
    if not 1 <= nat <= _lib.EPW_MAX_ATOMS:
        raise ValueError("polar: 1..%d atoms" % _lib.EPW_MAX_ATOMS)
    p = _lib.EpwPolar()
    p.nat = nat
    p.vectors[:] = list(np.asarray(vectors, dtype=np.float64).reshape(9))
    t = np.zeros((_lib.EPW_MAX_ATOMS, 3))
    t[:nat] = tau
    p.tau[:] = list(t.reshape(-1))
    z = np.zeros((_lib.EPW_MAX_ATOMS, 3, 3))
    z[:nat] = np.asarray(zstar, dtype=np.float64)
    p.zstar[:] = list(z.reshape(-1))
    p.eps_inf[:] = list(np.asarray(eps_inf, dtype=np.float64).reshape(9))
    m = np.ones(_lib.EPW_MAX_ATOMS)
    m[:nat] = np.asarray(masses, dtype=np.float64)
    p.mass[:] = list(m)
    p.prefactor, p.alpha, p.cutoff = float(prefactor), float(alpha), float(cutoff)
    return p


class Points:
    """Device-resident fine points: k set, q set, optional k+q map and
    optional given phonon states."""

    def __init__(self, kfrac, qfrac, kq=None, omega=None, evec=None, device="cuda"):
        d = torch.device(device)
        self.k = _dev(kfrac, torch.float64, d)
        self.q = _dev(qfrac, torch.float64, d)
        self.kq = None if kq is None else _dev(kq, torch.int32, d)
        self.omega = None if omega is None else _dev(omega, torch.float64, d)
        self.evec = None if evec is None else _dev(evec, torch.complex128, d)

    def c_struct(self):
        return _lib.EpwPoints(self.k.shape[0], self.q.shape[0], _ptr(self.k), _ptr(self.q),
                              _ptr(self.kq), _ptr(self.omega), _ptr(self.evec))


ORDERS = {"auto": 0, "k_inner": 1, "k_outer": 2}


def make_params(T=300.0, mu=0.0, sigma=0.05, omega_cut=1e-3, deg_tol=1e-6, nq_norm=0.0,
                dtype="fp64", chunk_q=0, accumulate=False, order="auto"):
    return _lib.EpwParams(float(T), float(mu), float(sigma), float(omega_cut), float(deg_tol),
                          float(nq_norm), DTYPES[dtype] if isinstance(dtype, str) else int(dtype),
                          int(chunk_q), int(bool(accumulate)), ORDERS[order] if isinstance(order, str) else int(order))


def epw_workspace_size(which, system, points, params):
    lib = _lib.load()
    s, p = system.c_struct(), points.c_struct()
    n = lib.epw_workspace_size(which, ctypes.byref(s), ctypes.byref(p), ctypes.byref(params))
    if n == 0:
        msg = lib.epw_last_error()
        raise EpwError(_lib.EPW_EINVAL, msg.decode() if msg else "")
    return int(n)


class Workspace:
    """Grow-only device workspace reused across calls on one stream."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf = None

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf


def epw_check_inputs(system, points, herm_tol=1e-12, workspace=None):
    """Validate the device arrays of a system and point set (synchronous);
    raises EpwError with the code of the first failed check."""
    lib = _lib.load()
    ws = workspace or Workspace(system.device)
    buf = ws.get(epw_workspace_size(EPW_WS_CHECK, system, points, make_params()))
    s, p = system.c_struct(), points.c_struct()
    _lib.check(lib.epw_check_inputs(ctypes.byref(s), ctypes.byref(p), float(herm_tol), _ptr(buf), buf.numel(),
                                    _stream(system.device)))


def epw_interp_g(system, points, params, workspace=None):
    """g_mn,nu(k,q) [nk][nq][nm][nb][nb] complex128 (materialised)."""
    lib = _lib.load()
    ws = workspace or Workspace(system.device)
    nbytes = epw_workspace_size(EPW_WS_INTERP_G, system, points, params)
    buf = ws.get(nbytes)
    nk, nq = points.k.shape[0], points.q.shape[0]
    out = torch.empty((nk, nq, system.nm, system.nb, system.nb), dtype=torch.complex128,
                      device=system.device)
    s, p = system.c_struct(), points.c_struct()
    _lib.check(lib.epw_interp_g(ctypes.byref(s), ctypes.byref(p), ctypes.byref(params), _ptr(out),
                                _ptr(buf), buf.numel(), _stream(system.device)))
    return out


def epw_imsigma(system, points, params, out=None, workspace=None):
    """Im Sigma_nk [nk][nb] float64 (Sec. 3 Eq. (8))."""
    lib = _lib.load()
    ws = workspace or Workspace(system.device)
    nbytes = epw_workspace_size(EPW_WS_IMSIGMA, system, points, params)
    buf = ws.get(nbytes)
    if out is None:
        out = torch.empty((points.k.shape[0], system.nb), dtype=torch.float64, device=system.device)
    s, p = system.c_struct(), points.c_struct()
    _lib.check(lib.epw_imsigma(ctypes.byref(s), ctypes.byref(p), ctypes.byref(params), _ptr(out),
                               _ptr(buf), buf.numel(), _stream(system.device)))
    return out


def epw_imsigma_noalloc(system, points, params, out=None):
    """Im Sigma_nk [nk][nb] float64 as epw_imsigma, with the library's own
    static device scratch instead of a workspace (no allocation in the call)."""
    lib = _lib.load()
    if out is None:
        out = torch.empty((points.k.shape[0], system.nb), dtype=torch.float64, device=system.device)
    s, p = system.c_struct(), points.c_struct()
    _lib.check(lib.epw_imsigma_noalloc(ctypes.byref(s), ctypes.byref(p), ctypes.byref(params), _ptr(out),
                                       _stream(system.device)))
    return out


def epw_resigma(system, points, params, want_tilde=True, workspace=None):
    """(Sigma'_nk on shell, Sigma~'_nk or None) [nk][nb] float64: the real part
    of Sec. 3 Eq. (3) at omega = eps_nk - eps_F and its Eq. (5) form."""
    lib = _lib.load()
    ws = workspace or Workspace(system.device)
    nbytes = epw_workspace_size(EPW_WS_RESIGMA, system, points, params)
    buf = ws.get(nbytes)
    d = system.device
    shape = (points.k.shape[0], system.nb)
    shell = torch.empty(shape, dtype=torch.float64, device=d)
    tilde = torch.empty(shape, dtype=torch.float64, device=d) if want_tilde else None
    s, p = system.c_struct(), points.c_struct()
    _lib.check(lib.epw_resigma(ctypes.byref(s), ctypes.byref(p), ctypes.byref(params), _ptr(shell), _ptr(tilde),
                               _ptr(buf), buf.numel(), _stream(d)))
    return shell, tilde


def epw_selfenergy_omega(system, points, params, wgrid, out=None, out0=None, workspace=None):
    """(Sigma_nk(omega) [nk][nb][nw] complex128, Sigma_nk(0) [nk][nb]
    complex128): the complex self-energy of Sec. 3 Eq. (3) at the frequencies
    wgrid (eV from eps_F), delta = params.sigma."""
    lib = _lib.load()
    ws = workspace or Workspace(system.device)
    d = system.device
    w = _dev(wgrid, torch.float64, d).contiguous()
    nw = w.shape[0]
    s, p = system.c_struct(), points.c_struct()
    nbytes = lib.epw_workspace_size_omega(ctypes.byref(s), ctypes.byref(p), ctypes.byref(params), nw)
    if nbytes == 0:
        msg = lib.epw_last_error()
        raise EpwError(_lib.EPW_EINVAL, msg.decode() if msg else "")
    buf = ws.get(nbytes)
    nk, nb = points.k.shape[0], system.nb
    if out is None:
        out = torch.empty((nk, nb, nw), dtype=torch.complex128, device=d)
    if out0 is None:
        out0 = torch.empty((nk, nb), dtype=torch.complex128, device=d)
    _lib.check(lib.epw_selfenergy_omega(ctypes.byref(s), ctypes.byref(p), ctypes.byref(params), nw, _ptr(w),
                                        _ptr(out), _ptr(out0), _ptr(buf), buf.numel(), _stream(d)))
    return out, out0


def epw_spectral_function(eps, mu, wgrid, sigma_w, sigma0):
    """A_nk(omega) [nk][nb][nw] float64 of Sec. 3 Eq. (10) from the output of
    epw_selfenergy_omega and the band energies eps [nk][nb] at the k points."""
    lib = _lib.load()
    d = sigma_w.device
    eps = _dev(eps, torch.float64, d).contiguous()
    w = _dev(wgrid, torch.float64, d).contiguous()
    nk, nb, nw = sigma_w.shape
    A = torch.empty((nk, nb, nw), dtype=torch.float64, device=d)
    _lib.check(lib.epw_spectral_function(nk, nb, nw, _ptr(eps), float(mu), _ptr(w), _ptr(sigma_w.contiguous()),
                                         _ptr(sigma0.contiguous()), _ptr(A), _stream(d)))
    return A


def spectral_function(system, points, params, wgrid, workspace=None):
    """(A [nk][nb][nw], Sigma(omega), Sigma(0), eps_k): Eq. (3) on the grid,
    then Eq. (10) with the band energies at the k points."""
    sig, sig0 = epw_selfenergy_omega(system, points, params, wgrid, workspace=workspace)
    eps, _ = epw_interp_bands(system.HR, system.Re, system.ndeg_e, points.k)
    return epw_spectral_function(eps, params.mu, wgrid, sig, sig0), sig, sig0, eps


def _host9(vectors):
    v = np.ascontiguousarray(np.asarray(vectors, dtype=np.float64).reshape(9))
    return v, v.ctypes.data_as(ctypes.c_void_p)


def epw_band_velocities(HR, R, ndeg, vectors, kfrac, deg_tol=1e-6):
    """(eps [nk][nb], U [nk][nb][nb], v [nk][nb][3]) on the device of HR."""
    lib = _lib.load()
    dev = HR.device
    HR = _dev(HR, torch.complex128, dev)
    R = _dev(R, torch.int32, dev)
    ndeg = _dev(ndeg, torch.int32, dev)
    k = _dev(kfrac, torch.float64, dev)
    nb, nk = HR.shape[-1], k.shape[0]
    eps = torch.empty((nk, nb), dtype=torch.float64, device=dev)
    U = torch.empty((nk, nb, nb), dtype=torch.complex128, device=dev)
    v = torch.empty((nk, nb, 3), dtype=torch.float64, device=dev)
    keep, vp = _host9(vectors)
    _lib.check(lib.epw_band_velocities(nb, R.shape[0], _ptr(R), _ptr(ndeg), _ptr(HR), vp, nk, _ptr(k),
                                       float(deg_tol), _ptr(eps), _ptr(U), _ptr(v), _stream(dev)))
    return eps, U, v


def epw_transport_coupling(system, points, params, vectors, want_lambda=True, want_pi=False, workspace=None):
    """(lambda_tr [nq][nm], lambda or None, Pi'' or None), Sec. 6 Eq. (55)."""
    lib = _lib.load()
    ws = workspace or Workspace(system.device)
    nbytes = epw_workspace_size(EPW_WS_TRANSPORT, system, points, params)
    buf = ws.get(nbytes)
    d = system.device
    shape = (points.q.shape[0], system.nm)
    ltr = torch.empty(shape, dtype=torch.float64, device=d)
    lam = torch.empty(shape, dtype=torch.float64, device=d) if want_lambda else None
    pi = torch.empty(shape, dtype=torch.float64, device=d) if want_pi else None
    keep, vp = _host9(vectors)
    s, p = system.c_struct(), points.c_struct()
    _lib.check(lib.epw_transport_coupling(ctypes.byref(s), ctypes.byref(p), ctypes.byref(params), vp, _ptr(ltr),
                                          _ptr(lam), _ptr(pi), _ptr(buf), buf.numel(), _stream(d)))
    return ltr, lam, pi


def epw_eliashberg_function(omega, lam, wgrid, sigma, nq_norm=None):
    """alpha^2 F on the grid (Eq. (12), or Eq. (54) from lambda_tr)."""
    lib = _lib.load()
    d = lam.device
    om = _dev(omega, torch.float64, d)
    lam = _dev(lam, torch.float64, d)
    w = _dev(wgrid, torch.float64, d)
    nq, nm = om.shape
    out = torch.empty(w.shape[0], dtype=torch.float64, device=d)
    _lib.check(lib.epw_eliashberg_function(nq, nm, _ptr(om), _ptr(lam), float(nq if nq_norm is None else nq_norm),
                                           w.shape[0], _ptr(w), float(sigma), _ptr(out), _stream(d)))
    return out


def epw_ziman_resistivity(wgrid, a2f_tr, temperatures):
    """rho(T) n e^2 / m_e of Eq. (53) for each temperature (K)."""
    lib = _lib.load()
    d = a2f_tr.device
    w = _dev(wgrid, torch.float64, d)
    a = _dev(a2f_tr, torch.float64, d)
    T = _dev(temperatures, torch.float64, d)
    out = torch.empty(T.shape[0], dtype=torch.float64, device=d)
    _lib.check(lib.epw_ziman_resistivity(w.shape[0], _ptr(w), _ptr(a), T.shape[0], _ptr(T), _ptr(out), _stream(d)))
    return out


def epw_phonon_selfenergy(system, points, params, want_lambda=True, workspace=None):
    """(Pi''_q,nu [nq][nm], lambda_q,nu [nq][nm] or None) float64: the phonon
    linewidth of Sec. 3 Eq. (9) on shell and the coupling strength of
    Sec. 3 Eq. (11)."""
    lib = _lib.load()
    ws = workspace or Workspace(system.device)
    nbytes = epw_workspace_size(EPW_WS_PHONON, system, points, params)
    buf = ws.get(nbytes)
    d = system.device
    nq, nm = points.q.shape[0], system.nm
    pi_im = torch.empty((nq, nm), dtype=torch.float64, device=d)
    lam = torch.empty((nq, nm), dtype=torch.float64, device=d) if want_lambda else None
    s, p = system.c_struct(), points.c_struct()
    _lib.check(lib.epw_phonon_selfenergy(ctypes.byref(s), ctypes.byref(p), ctypes.byref(params), _ptr(pi_im),
                                         _ptr(lam), _ptr(buf), buf.numel(), _stream(d)))
    return pi_im, lam


def epw_imsigma_backward(system, points, params, w, want=("gR", "HR", "omega"), workspace=None):
    """(dL/dgR, dL/dHR, dL/domega) for L = sum w Im Sigma."""
    lib = _lib.load()
    ws = workspace or Workspace(system.device)
    nbytes = epw_workspace_size(EPW_WS_IMSIGMA_BACKWARD, system, points, params)
    buf = ws.get(nbytes)
    d = system.device
    w = _dev(w, torch.float64, d)
    dg = torch.empty_like(system.gR) if "gR" in want else None
    dh = torch.empty_like(system.HR) if "HR" in want else None
    nq, nm = points.q.shape[0], system.nm
    dom = torch.empty((nq, nm), dtype=torch.float64, device=d) if "omega" in want else None
    s, p = system.c_struct(), points.c_struct()
    _lib.check(lib.epw_imsigma_backward(ctypes.byref(s), ctypes.byref(p), ctypes.byref(params),
                                        _ptr(w), _ptr(dg), _ptr(dh), _ptr(dom), _ptr(buf), buf.numel(),
                                        _stream(d)))
    return dg, dh, dom


def epw_timing_enable(on=True):
    _lib.check(_lib.load().epw_timing_enable(1 if on else 0))


def epw_timing_read(stage):
    """(total milliseconds, launches) recorded for a stage since the last read."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _lib.check(_lib.load().epw_timing_read(int(stage), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value
