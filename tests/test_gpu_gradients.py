"""Hand-written adjoint of L = sum w Im Sigma against the FP64 CPU reference
gradient (torch autograd of the oracle forward) and central finite
differences of the HIP forward; tolerance 1e-6 relative (infinity norm over
all entries for the reference, over the checked entries for FD)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from oracle import interp, lattice, torch_ref
from paper_1604_03525_amd import _lib, autograd, epw
from paper_1604_03525_amd import inputs as I
from tests.helpers import fcc_small_case, rel_err, toy_case

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _setup(c, kg):
    om, ev = interp.phonons(c["DR"], c["R"], c["nd"], c["q"])      # oracle phonon states
    w = I.loss_weights(len(c["k"]), c["HR"].shape[1], 1)
    kw = dict(Re=c["R"], ndeg_e=c["nd"], Rp=c["R"], ndeg_p=c["nd"], kpoints=c["k"], qpoints=c["q"],
              kq=c["kq"], T=c["T"], mu=c["mu"], sigma=c["sigma"])
    return om, ev, w, kw


def _hip_grads(c, om, ev, w, dtype="fp64"):
    g = torch.tensor(c["gR"], device=DEV, requires_grad=True)
    h = torch.tensor(c["HR"], device=DEV, requires_grad=True)
    o = torch.tensor(om, device=DEV, requires_grad=True)
    ims = autograd.imsigma(g, h, o, torch.as_tensor(ev).to(DEV), c["R"], c["nd"], c["R"], c["nd"], c["k"], c["q"],
                           c["kq"], T=c["T"], mu=c["mu"], sigma=c["sigma"], dtype=dtype)
    L = torch.sum(torch.as_tensor(w, device=DEV) * ims)
    L.backward()
    return float(L.detach()), g.grad.cpu().numpy(), h.grad.cpu().numpy(), o.grad.cpu().numpy()


@pytest.mark.parametrize("case", ["toy12", "fcc3"])
def test_adjoint_matches_reference_gradient(case):
    if case == "toy12":
        c = toy_case((12, 12, 12))          # the differentiation workload: 12^3 k x 12^3 q
    else:
        c = fcc_small_case(nb=3, kg=(3, 3, 3))
    _say("gradients", case)
    om, ev, w, kw = _setup(c, None)
    L_ref, ims_ref, dg_ref, dh_ref, dom_ref = torch_ref.loss_and_grads(c["gR"], c["HR"], om, ev, w, **kw)
    L, dg, dh, dom = _hip_grads(c, om, ev, w)
    _say("  L", L, L_ref, "rel errs g/h/omega", rel_err(dg, dg_ref), rel_err(dh, dh_ref), rel_err(dom, dom_ref))
    assert abs(L - L_ref) < 1e-10 * abs(L_ref)
    assert rel_err(dg, dg_ref) < 1e-6
    assert rel_err(dh, dh_ref) < 1e-6
    assert rel_err(dom, dom_ref) < 1e-6
    # Euler: L is homogeneous of degree 2 in g
    assert abs(np.sum(np.real(np.conj(dg) * c["gR"])) - 2 * L) < 1e-9 * abs(L)


def test_adjoint_finite_differences_toy12():
    """Central differences (h = 1e-6) of the HIP forward on 64 random entries
    per gradient (entries from seed 4)."""
    c = toy_case((12, 12, 12))
    om, ev, w, kw = _setup(c, None)
    L0, dg, dh, dom = _hip_grads(c, om, ev, w)
    sysd_cache = {}
    pts = epw.Points(c["k"], c["q"], c["kq"], omega=om, evec=ev, device=DEV)
    par = epw.make_params(T=c["T"], mu=c["mu"], sigma=c["sigma"])
    wt = torch.as_tensor(w, device=DEV)
    ws = epw.Workspace(DEV)

    def loss(g=None, h=None, o=None):
        s = epw.System(c["R"], c["nd"], c["R"], c["nd"], c["HR"] if h is None else h, None,
                       c["gR"] if g is None else g, DEV)
        p = pts if o is None else epw.Points(c["k"], c["q"], c["kq"], omega=o, evec=ev, device=DEV)
        return float(torch.sum(wt * epw.epw_imsigma(s, p, par, workspace=ws)))

    rng = np.random.default_rng(4)
    hs = 1e-6
    _say("FD gR")
    worst = 0.0
    flat = c["gR"].reshape(-1)
    for idx in rng.choice(flat.size, 64, replace=False):
        for unit in (1.0, 1j):
            gp = flat.copy(); gp[idx] += hs * unit
            gm = flat.copy(); gm[idx] -= hs * unit
            fd = (loss(g=gp.reshape(c["gR"].shape)) - loss(g=gm.reshape(c["gR"].shape))) / (2 * hs)
            an = dg.reshape(-1)[idx]
            an = an.real if unit == 1.0 else an.imag
            worst = max(worst, abs(fd - an))
    assert worst < 1e-6 * np.abs(dg).max(), worst / np.abs(dg).max()
    _say("FD HR")
    worst = 0.0
    flatH = c["HR"].reshape(-1)
    for idx in rng.choice(flatH.size, min(64, flatH.size), replace=False):
        for unit in (1.0, 1j):
            hp = flatH.copy(); hp[idx] += hs * unit
            hm = flatH.copy(); hm[idx] -= hs * unit
            fd = (loss(h=hp.reshape(c["HR"].shape)) - loss(h=hm.reshape(c["HR"].shape))) / (2 * hs)
            an = dh.reshape(-1)[idx]
            an = an.real if unit == 1.0 else an.imag
            worst = max(worst, abs(fd - an))
    assert worst < 1e-6 * np.abs(dh).max(), worst / np.abs(dh).max()
    _say("FD omega")
    worst = 0.0
    kept = np.flatnonzero(om.reshape(-1) >= 2e-3)
    for idx in rng.choice(kept, 64, replace=False):
        op = om.reshape(-1).copy(); op[idx] += hs
        omn = om.reshape(-1).copy(); omn[idx] -= hs
        fd = (loss(o=op.reshape(om.shape)) - loss(o=omn.reshape(om.shape))) / (2 * hs)
        worst = max(worst, abs(fd - dom.reshape(-1)[idx]))
    assert worst < 1e-6 * np.abs(dom).max(), worst / np.abs(dom).max()


def test_adjoint_chunking_and_accumulate():
    """q chunks of 5 and the accumulate flag give the same gradients."""
    c = fcc_small_case(nb=2, kg=(3, 3, 3), seed=5)
    om, ev, w, kw = _setup(c, None)
    sysd = epw.System(c["R"], c["nd"], c["R"], c["nd"], c["HR"], None, c["gR"], DEV)
    pts = epw.Points(c["k"], c["q"], c["kq"], omega=om, evec=ev, device=DEV)
    a = epw.epw_imsigma_backward(sysd, pts, epw.make_params(T=c["T"], mu=c["mu"], sigma=c["sigma"]), w)
    b = epw.epw_imsigma_backward(sysd, pts, epw.make_params(T=c["T"], mu=c["mu"], sigma=c["sigma"], chunk_q=5), w)
    for x, y in zip(a, b):
        assert rel_err(y.cpu().numpy(), x.cpu().numpy()) < 1e-12


@pytest.mark.parametrize("case", ["toy12", "fcc3"])
def test_adjoint_fp32_matches_reference_gradient(case):
    """The float32 adjoint (complex64 contractions, rotations and per-pair
    adjoint; float64 eigen-adjoint and outputs) against the FP64 reference
    gradient.  Tolerance 1e-4 relative: float32 rounding (6e-8) grown by the
    contraction lengths (N_e, N_k up to ~1.7e3 terms) and by the forward's own
    float32 error, which enters every weight of the adjoint."""
    if case == "toy12":
        c = toy_case((12, 12, 12))
    else:
        c = fcc_small_case(nb=3, kg=(3, 3, 3))
    om, ev, w, kw = _setup(c, None)
    L_ref, ims_ref, dg_ref, dh_ref, dom_ref = torch_ref.loss_and_grads(c["gR"], c["HR"], om, ev, w, **kw)
    L, dg, dh, dom = _hip_grads(c, om, ev, w, dtype="fp32")
    _say("fp32 gradients", case, "rel errs L/g/h/omega", abs(L - L_ref) / abs(L_ref), rel_err(dg, dg_ref),
         rel_err(dh, dh_ref), rel_err(dom, dom_ref))
    assert abs(L - L_ref) < 1e-5 * abs(L_ref)
    assert rel_err(dg, dg_ref) < 1e-4
    assert rel_err(dh, dh_ref) < 1e-4
    assert rel_err(dom, dom_ref) < 1e-4


@pytest.mark.parametrize("case", ["toy12", "fcc3"])
def test_adjoint_split_bf16_matches_reference_gradient(case):
    """The split-bf16 adjoint (the R_e <-> k contractions, recompute and
    adjoint, on bf16 hi + lo planes with float32 accumulation; everything
    else as the float32 adjoint) against the FP64 reference gradient.
    Tolerance 1e-4 relative, the bar of the split-bf16 forward: dropping
    lo.lo leaves about 2^-16 = 1.5e-5 relative per product, which the float32
    sums over N_e and N_k terms and the forward's own error (it sets every
    weight of the adjoint) grow by a small factor."""
    if case == "toy12":
        c = toy_case((12, 12, 12))
    else:
        c = fcc_small_case(nb=3, kg=(3, 3, 3))
    om, ev, w, kw = _setup(c, None)
    L_ref, ims_ref, dg_ref, dh_ref, dom_ref = torch_ref.loss_and_grads(c["gR"], c["HR"], om, ev, w, **kw)
    L, dg, dh, dom = _hip_grads(c, om, ev, w, dtype="split_bf16")
    errs = (abs(L - L_ref) / abs(L_ref), rel_err(dg, dg_ref), rel_err(dh, dh_ref), rel_err(dom, dom_ref))
    _say("split-bf16 gradients", case, "rel errs L/g/h/omega", *errs)
    assert errs[0] < 1e-4
    assert max(errs[1:]) < 1e-4


def test_adjoint_fp32_chunking_accumulate():
    """float32 and split-bf16: chunks of 5 q give the result of one chunk (to
    float32 rounding), accumulate adds onto the outputs."""
    c = fcc_small_case(nb=2, kg=(3, 3, 3), seed=5)
    om, ev, w, kw = _setup(c, None)
    sysd = epw.System(c["R"], c["nd"], c["R"], c["nd"], c["HR"], None, c["gR"], DEV)
    pts = epw.Points(c["k"], c["q"], c["kq"], omega=om, evec=ev, device=DEV)
    mk = lambda **kw2: epw.make_params(T=c["T"], mu=c["mu"], sigma=c["sigma"], dtype="fp32", **kw2)
    a = epw.epw_imsigma_backward(sysd, pts, mk(), w)
    b = epw.epw_imsigma_backward(sysd, pts, mk(chunk_q=5), w)
    for x, y in zip(a, b):
        assert rel_err(y.cpu().numpy(), x.cpu().numpy()) < 1e-5
    ref = epw.epw_imsigma_backward(sysd, pts, epw.make_params(T=c["T"], mu=c["mu"], sigma=c["sigma"]), w)
    for x, y in zip(a, ref):
        assert rel_err(x.cpu().numpy(), y.cpu().numpy()) < 1e-4
    mb = lambda **kw2: epw.make_params(T=c["T"], mu=c["mu"], sigma=c["sigma"], dtype="split_bf16", **kw2)
    a = epw.epw_imsigma_backward(sysd, pts, mb(), w)
    b = epw.epw_imsigma_backward(sysd, pts, mb(chunk_q=5), w)
    for x, y in zip(a, b):
        assert rel_err(y.cpu().numpy(), x.cpu().numpy()) < 1e-5
    for x, y in zip(a, ref):
        assert rel_err(x.cpu().numpy(), y.cpu().numpy()) < 1e-4
    acc = epw.make_params(T=c["T"], mu=c["mu"], sigma=c["sigma"], dtype="split_bf16", accumulate=True)
    lib = _lib.load()
    outs = [t.clone() for t in a]
    s_, p_ = sysd.c_struct(), pts.c_struct()
    ws = epw.Workspace(DEV)
    buf = ws.get(epw.epw_workspace_size(epw.EPW_WS_IMSIGMA_BACKWARD, sysd, pts, acc))
    wt = torch.as_tensor(w, device=DEV)
    _lib.check(lib.epw_imsigma_backward(ctypes.byref(s_), ctypes.byref(p_), ctypes.byref(acc), ctypes.c_void_p(
        wt.data_ptr()), ctypes.c_void_p(outs[0].data_ptr()), ctypes.c_void_p(outs[1].data_ptr()),
        ctypes.c_void_p(outs[2].data_ptr()), ctypes.c_void_p(buf.data_ptr()), buf.numel(),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    for x, y in zip(outs, a):
        assert rel_err(x.cpu().numpy(), 2 * y.cpu().numpy()) < 1e-6
