"""The R_e <-> k sums of the FP64 and FP32 paths run over the pairs (R, -R) of
the R_e list (c B+ + i s B- per pair); a vector without its negative, the
zero vector and a vector listed twice enter unpaired.  These cases break the
symmetry of a Wigner-Seitz list on purpose: the forward is compared with the
oracle (grid runs, where k+q is a member of the k set) at the precisions'
parity tolerances (FP64 1e-10, FP32 1e-5), the adjoint with the torch
reference gradient (1e-6)."""
import sys

import numpy as np
import pytest
import torch

from oracle import interp, selfenergy as se, torch_ref
from paper_1604_03525_amd import autograd, epw
from paper_1604_03525_amd import inputs as I
from tests.helpers import fcc_small_case, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _asymmetric_case(nb=3, seed=5):
    """fcc_small_case with three vectors removed (their negatives stay, now
    without a partner) and one vector appended a second time with its own,
    rescaled data; the same list serves R_e and R_p."""
    c = fcc_small_case(nb=nb, kg=(3, 3, 3), seed=seed)
    R, nd = c["R"], c["nd"]
    zero = int(np.flatnonzero(np.all(R == 0, axis=1))[0])
    nonzero = [i for i in range(len(R)) if i != zero]
    drop = set(nonzero[1:8:3])                      # three non-zero vectors
    keep = [i for i in range(len(R)) if i not in drop]
    dup = nonzero[0]
    idx = np.array(keep + [dup])
    c2 = dict(c)
    c2["R"] = np.ascontiguousarray(R[idx])
    c2["nd"] = np.ascontiguousarray(nd[idx])
    c2["HR"] = np.ascontiguousarray(c["HR"][idx])
    c2["HR"][-1] *= 0.5
    c2["DR"] = np.ascontiguousarray(c["DR"][idx])
    c2["DR"][-1] *= 0.5
    g = c["gR"][idx][:, idx]
    g[-1] *= 0.5
    c2["gR"] = np.ascontiguousarray(g)
    # the list is no longer closed under R -> -R
    rows = {tuple(r) for r in c2["R"]}
    assert any(tuple(-r) not in rows for r in c2["R"])
    return c2


@pytest.mark.parametrize("dtype,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_folded_forward_any_r_list(dtype, tol):
    c = _asymmetric_case()
    _say("folded forward, asymmetric R list", dtype, len(c["R"]), "vectors")
    sysd = epw.System(c["R"], c["nd"], c["R"], c["nd"], c["HR"], c["DR"], c["gR"], DEV)
    pts = epw.Points(c["k"], c["q"], c["kq"], device=DEV)
    par = epw.make_params(T=c["T"], mu=c["mu"], sigma=c["sigma"], dtype=dtype)
    ims = epw.epw_imsigma(sysd, pts, par).cpu().numpy()
    ref = se.imsigma(c["HR"], c["R"], c["nd"], c["DR"], c["R"], c["nd"], c["gR"], c["k"], c["q"],
                     c["T"], c["mu"], c["sigma"])
    err = rel_err(ims, ref)
    _say("  rel err", err)
    assert np.max(np.abs(ref)) > 0
    assert err < tol


def test_folded_adjoint_any_r_list():
    c = _asymmetric_case()
    _say("folded adjoint, asymmetric R list", len(c["R"]), "vectors")
    om, ev = interp.phonons(c["DR"], c["R"], c["nd"], c["q"])
    w = I.loss_weights(len(c["k"]), c["HR"].shape[1], 1)
    kw = dict(Re=c["R"], ndeg_e=c["nd"], Rp=c["R"], ndeg_p=c["nd"], kpoints=c["k"], qpoints=c["q"],
              kq=c["kq"], T=c["T"], mu=c["mu"], sigma=c["sigma"])
    L_ref, _, dg_ref, dh_ref, dom_ref = torch_ref.loss_and_grads(c["gR"], c["HR"], om, ev, w, **kw)
    g = torch.tensor(c["gR"], device=DEV, requires_grad=True)
    h = torch.tensor(c["HR"], device=DEV, requires_grad=True)
    o = torch.tensor(om, device=DEV, requires_grad=True)
    ims = autograd.imsigma(g, h, o, torch.as_tensor(ev).to(DEV), c["R"], c["nd"], c["R"], c["nd"], c["k"], c["q"],
                           c["kq"], T=c["T"], mu=c["mu"], sigma=c["sigma"], dtype="fp64")
    L = torch.sum(torch.as_tensor(w, device=DEV) * ims)
    L.backward()
    dg, dh, dom = g.grad.cpu().numpy(), h.grad.cpu().numpy(), o.grad.cpu().numpy()
    Lv = float(L.detach())
    _say("  L", Lv, L_ref, "rel errs g/h/omega", rel_err(dg, dg_ref), rel_err(dh, dh_ref), rel_err(dom, dom_ref))
    assert abs(Lv - L_ref) < 1e-10 * abs(L_ref)
    assert rel_err(dg, dg_ref) < 1e-6
    assert rel_err(dh, dh_ref) < 1e-6
    assert rel_err(dom, dom_ref) < 1e-6
