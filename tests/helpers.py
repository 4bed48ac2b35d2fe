"""Shared builders for the GPU parity tests: the same seeded inputs go to
the HIP library and to the oracle."""
import numpy as np

from oracle import lattice
from paper_1604_03525_amd import inputs as I


def rel_err(x, ref):
    """Infinity-norm relative error max|x - ref| / max|ref|."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(x - ref)) / (den if den > 0 else 1.0))


def toy_case(kg=(8, 8, 8), qg=None):
    qg = kg if qg is None else qg
    m = I.toy_model(kg, qg)
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    HR, DR, gR = I.toy_arrays(R, R)
    k = lattice.grid_points(*kg)
    q = lattice.grid_points(*qg)
    kq = lattice.kq_index(kg, qg)
    return dict(model=m, R=R, nd=nd, HR=HR, DR=DR, gR=gR, k=k, q=q, kq=kq,
                T=m.T, mu=m.mu, sigma=m.sigma)


def fcc_small_case(nb=3, kg=(4, 4, 4), coarse=(2, 2, 2), seed=1, natoms=2):
    R, nd = lattice.ws_vectors(I.FCC_METRIC, coarse)
    atoms = I.ATOMS_FCC2 if natoms == 2 else I.ATOMS_FCC3
    nm = 3 * natoms
    HR = I.random_hamiltonian(R, I.FCC_VECTORS, nb, seed=seed, scale=0.8)
    DR = I.spring_dynmat(R, I.FCC_VECTORS, atoms, shells=2, seed=seed + 1, scale=4e-4)
    gR = I.random_vertex(R, R, I.FCC_VECTORS, nm, nb, seed=seed + 2, g0=0.05)
    k = lattice.grid_points(*kg)
    kq = lattice.kq_index(kg, kg)
    return dict(R=R, nd=nd, HR=HR, DR=DR, gR=gR, k=k, q=k, kq=kq, T=300.0, mu=0.1, sigma=0.15)


def realistic_case():
    m = I.realistic_model()
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    HR, DR, gR = I.realistic_arrays(R, R)
    k = lattice.grid_points(*m.kgrid)
    kq = lattice.kq_index(m.kgrid, m.qgrid)
    return dict(model=m, R=R, nd=nd, HR=HR, DR=DR, gR=gR, k=k, q=k, kq=kq,
                T=m.T, mu=m.mu, sigma=m.sigma)


def mobility_small_case(coarse=(3, 3, 3), nk=24, nq=40, nb=16, seed=20):
    """The mobility-scale system's shape (fcc, 3 atoms, 16 bands, 9 modes,
    random k and q, off-grid k+q) on a small coarse grid so the oracle can
    evaluate it completely."""
    R, nd = lattice.ws_vectors(I.FCC_METRIC, coarse)
    HR = I.random_hamiltonian(R, I.FCC_VECTORS, nb, seed=seed, decay=1.5, scale=0.6)
    DR = I.spring_dynmat(R, I.FCC_VECTORS, I.ATOMS_FCC3, shells=2, seed=seed + 1, scale=4e-4)
    gR = I.random_vertex(R, R, I.FCC_VECTORS, 9, nb, seed=seed + 2, g0=0.05)
    k = I.random_points(nk, 3)
    q = I.random_points(nq, 2)
    return dict(R=R, nd=nd, HR=HR, DR=DR, gR=gR, k=k, q=q, kq=None, T=300.0, mu=0.0, sigma=0.1)
