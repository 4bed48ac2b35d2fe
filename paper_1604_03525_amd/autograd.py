"""torch.autograd binding of Im Sigma_nk and its hand-written adjoint.

    ims = imsigma(gR, HR, omega, evec, Re, ndeg_e, Rp, ndeg_p, kfrac, qfrac, kq, ...)
    (w * ims).sum().backward()      # gR.grad, HR.grad, omega.grad

forward -> epw_imsigma, backward -> epw_imsigma_backward with the incoming
gradient as the loss weights w_nk.  The phonon eigenvectors evec are held
fixed, so omega.grad is the partial derivative at fixed e_q.  Complex
gradients follow torch's convention (dL/dRe + i dL/dIm).  With `polar` (the
data of epw.make_polar) the vertex carries the long-range term of Sec. 4 in
both directions.
"""
import torch

from . import epw


class ImSigmaFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gR, HR, omega, evec, Re, ndeg_e, Rp, ndeg_p, points_k, points_q, kq, params, workspace, polar):
        sysd = epw.System(Re, ndeg_e, Rp, ndeg_p, HR, None, gR, gR.device, polar=polar)
        pts = epw.Points(points_k, points_q, kq, omega=omega, evec=evec, device=gR.device)
        out = epw.epw_imsigma(sysd, pts, params, workspace=workspace)
        ctx.sysd, ctx.pts, ctx.params, ctx.workspace = sysd, pts, params, workspace
        return out

    @staticmethod
    def backward(ctx, grad_out):
        want = []
        if ctx.needs_input_grad[0]:
            want.append("gR")
        if ctx.needs_input_grad[1]:
            want.append("HR")
        if ctx.needs_input_grad[2]:
            want.append("omega")
        dg, dh, dom = epw.epw_imsigma_backward(ctx.sysd, ctx.pts, ctx.params, grad_out.contiguous(),
                                               want=tuple(want), workspace=ctx.workspace)
        return (dg, dh, dom) + (None,) * 11


def imsigma(gR, HR, omega, evec, Re, ndeg_e, Rp, ndeg_p, kfrac, qfrac, kq, T=300.0, mu=0.0, sigma=0.05,
            omega_cut=1e-3, deg_tol=1e-6, nq_norm=0.0, dtype="fp64", chunk_q=0, workspace=None, polar=None):
    """Im Sigma_nk [nk][nb] as a differentiable function of gR, HR and omega
    (device tensors: gR, HR complex128; omega float64; evec complex128)."""
    params = epw.make_params(T=T, mu=mu, sigma=sigma, omega_cut=omega_cut, deg_tol=deg_tol, nq_norm=nq_norm,
                             dtype=dtype, chunk_q=chunk_q)
    ws = workspace or epw.Workspace(gR.device)
    return ImSigmaFn.apply(gR, HR, omega, evec, Re, ndeg_e, Rp, ndeg_p, kfrac, qfrac, kq, params, ws, polar)
