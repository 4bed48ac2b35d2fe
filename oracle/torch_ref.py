"""Reference gradient: the forward of Sec. 3 Eq. (8) written in plain torch
CPU float64 and differentiated by autograd.

Test infrastructure only (see oracle/__init__.py).

Loss L = sum_nk w_nk Im Sigma_nk (Im Sigma after the degenerate average).
The differentiable inputs are g(R_e,R_p) (complex), H(R_e) (complex) and
omega_q,nu (real); the phonon eigenvectors e_q are held fixed, so dL/domega
is the partial derivative at fixed e_q through the Bose factor, the
Gaussians and 1/sqrt(2 omega).  Complex gradients follow torch's convention
dL/dRe + i dL/dIm.  H(k) is the Hermitised sum, so every entry of every H(R)
is an independent complex parameter.

The contraction order here (R_p first for all q, then R_e for all k, then
gather of the k+q states from the k grid) differs on purpose from the NumPy
oracle's (R_e first per k, eigensolve at the unfolded k+q): the two forwards
cross-check each other.
"""
import math

import numpy as np
import torch

KB_EV = 8.617333262e-5


def _phases(points, R, ndeg):
    x = torch.as_tensor(np.asarray(points, dtype=np.float64)) @ \
        torch.as_tensor(np.asarray(R, dtype=np.float64)).T
    x = x - torch.floor(x + 0.5)
    return torch.exp(2j * math.pi * x.to(torch.complex128)) / \
        torch.as_tensor(np.asarray(ndeg, dtype=np.float64))[None, :]


def imsigma_torch(gR, HR, omega, evec, Re, ndeg_e, Rp, ndeg_p, kpoints, qpoints,
                  kq, T, mu, sigma, omega_cut=1e-3, deg_tol=1e-6, nq_norm=None, polar_lr=None):
    """Im Sigma [Nk][nb] as a differentiable torch function.

    gR [Ne][Np][nm][nb][nb] complex128, HR [Ne][nb][nb] complex128,
    omega [Nq][nm] float64, evec [Nq][nm][nm] complex128 (constant),
    kq [Nk][Nq] int: index of k+q in the k list (grid runs only).
    polar_lr [Nq][nm] complex (constant), optional: the long-range factor of
    Sec. 4 without its 1/sqrt(2 omega); the vertex then gains
    (polar_lr / sqrt(2 omega)) [U_k+q^dag U_k]_mn."""
    nq_norm = len(qpoints) if nq_norm is None else nq_norm
    ph_q = _phases(qpoints, Rp, ndeg_p)                        # [Q][Np]
    ph_k = _phases(kpoints, Re, ndeg_e)                        # [K][Ne]
    evec = torch.as_tensor(evec)
    kq = None if kq is None else torch.as_tensor(np.asarray(kq, dtype=np.int64))
    # R_p -> q, mode rotation with 1/sqrt(2 omega) (masked modes -> 0)
    gq = torch.einsum("qp,epaij->eqaij", ph_q, gR)
    keep = omega.detach() >= omega_cut
    safe = torch.where(keep, omega, torch.ones_like(omega))
    scale = torch.where(keep, 1.0 / torch.sqrt(2.0 * safe), torch.zeros_like(omega))
    gnu = torch.einsum("eqaij,qav->eqvij", gq, evec) * scale[None, :, :, None, None]
    # R_e -> k
    ne = gR.shape[0]
    gk = (ph_k @ gnu.reshape(ne, -1)).reshape((len(kpoints),) + gnu.shape[1:])
    # bands at k and (gathered) at k+q
    Hk = ph_k @ HR.reshape(ne, -1)
    nb = HR.shape[-1]
    Hk = Hk.reshape(-1, nb, nb)
    Hk = 0.5 * (Hk + Hk.conj().transpose(-1, -2))
    eps, U = torch.linalg.eigh(Hk)
    if kq is not None:
        eps_kq = eps[kq]                                       # [K][Q][nb]
        U_kq = U[kq]                                           # [K][Q][nb][nb]
    else:
        # off-grid: diagonalise H at every k+q
        kqp = (np.asarray(kpoints, dtype=np.float64)[:, None, :] +
               np.asarray(qpoints, dtype=np.float64)[None, :, :]).reshape(-1, 3)
        Hq = (_phases(kqp, Re, ndeg_e) @ HR.reshape(ne, -1)).reshape(-1, nb, nb)
        Hq = 0.5 * (Hq + Hq.conj().transpose(-1, -2))
        e2, U2 = torch.linalg.eigh(Hq)
        eps_kq = e2.reshape(len(kpoints), len(qpoints), nb)
        U_kq = U2.reshape(len(kpoints), len(qpoints), nb, nb)
    gb = torch.einsum("kqim,kqvij,kjn->kqvmn", U_kq.conj(), gk, U)
    if polar_lr is not None:
        ov = torch.einsum("kqim,kin->kqmn", U_kq.conj(), U)
        lr = torch.as_tensor(np.asarray(polar_lr, dtype=np.complex128)) * scale
        gb = gb + lr[None, :, :, None, None] * ov[:, :, None, :, :]
    # weights of Eq. (8)
    if T == 0.0:
        nB = torch.zeros_like(safe)
        f = torch.where(eps_kq < mu, 1.0, torch.where(eps_kq > mu, 0.0, 0.5))
    else:
        nB = 1.0 / torch.expm1(safe / (KB_EV * T))
        f = 1.0 / (torch.exp((eps_kq - mu) / (KB_EV * T)) + 1.0)
    nB = nB[None, :, :, None, None]
    f = f[:, :, None, :, None]
    x = eps[:, None, None, None, :] - eps_kq[:, :, None, :, None]
    w = safe[None, :, :, None, None]
    norm = 1.0 / (sigma * math.sqrt(math.pi))
    W = (nB + f) * torch.exp(-((x + w) / sigma) ** 2) * norm + \
        (nB + 1.0 - f) * torch.exp(-((x - w) / sigma) ** 2) * norm
    W = W * keep[None, :, :, None, None]
    ims = (math.pi / nq_norm) * torch.sum(torch.abs(gb) ** 2 * W, dim=(1, 2, 3))
    # degenerate average (groups fixed by the eigenvalues: no gradient path)
    e_np = eps.detach().numpy()
    groups = np.arange(nb)[None, :].repeat(len(kpoints), 0)
    for p in range(len(kpoints)):
        for n in range(1, nb):
            if abs(e_np[p, n] - e_np[p, n - 1]) < deg_tol:
                groups[p, n] = groups[p, n - 1]
    A = np.zeros((len(kpoints), nb, nb))
    for p in range(len(kpoints)):
        for n in range(nb):
            members = groups[p] == groups[p, n]
            A[p, n, members] = 1.0 / members.sum()
    return torch.einsum("pnm,pm->pn", torch.as_tensor(A), ims)


def loss_and_grads(gR, HR, omega, evec, w, **kw):
    """L = sum w * Im Sigma and its autograd gradients (dL/dgR, dL/dHR,
    dL/domega) as NumPy arrays."""
    g = torch.tensor(gR, dtype=torch.complex128, requires_grad=True)
    h = torch.tensor(HR, dtype=torch.complex128, requires_grad=True)
    om = torch.tensor(omega, dtype=torch.float64, requires_grad=True)
    ims = imsigma_torch(g, h, om, evec, **kw)
    L = torch.sum(torch.as_tensor(w) * ims)
    L.backward()
    return (float(L.detach()), ims.detach().numpy(), g.grad.numpy(), h.grad.numpy(),
            om.grad.numpy())
