"""Seeded synthetic inputs shaped after the paper's workloads.

This module draws random numbers and builds model real-space inputs
(H(R_e), D(R_p), g(R_e,R_p), point sets).  It holds no step of the method:
no Fourier sum, no eigensolve, no self-energy.  Both the HIP library's tests
and the FP64 oracle consume exactly these arrays.  The Wigner-Seitz vector
lists are arguments, produced by whichever side is being exercised (the two
implementations are bit-identical and tested to be).

The paper's own systems (SiC, Si, B-doped diamond, Pb, GaN, MgB2) need DFPT
data that is not available; these models stand in for them with the same
array shapes and the same structure: exponentially localised real-space
couplings, a random-phase vertex, Gamma-centred or uniformly random fine
points (Sec. 8 and Sec. 10.1-10.2 use both).

Energies are in eV, temperatures in K, lengths in units of the cubic
lattice constant a.
"""
from dataclasses import dataclass, field
import itertools

import numpy as np

# ---------------------------------------------------------------- lattices

SC_METRIC = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
FCC_METRIC = ((2, 1, 1), (1, 2, 1), (1, 1, 2))      # (a/2)^2 * this

SC_VECTORS = np.eye(3)
FCC_VECTORS = 0.5 * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])

ATOMS_SC1 = np.zeros((1, 3))
ATOMS_FCC2 = np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.25]])
ATOMS_FCC3 = np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.25], [-0.25, -0.25, -0.25]])


def cartesian(R, vectors):
    """Cartesian coordinates (units of a) of integer lattice vectors."""
    return np.asarray(R, dtype=np.float64) @ np.asarray(vectors, dtype=np.float64)


def _minus_index(R):
    pos = {tuple(int(x) for x in r): i for i, r in enumerate(np.asarray(R))}
    out = np.empty(len(R), dtype=np.int64)
    for i, r in enumerate(np.asarray(R)):
        key = tuple(-int(x) for x in r)
        if key not in pos:
            raise ValueError("vector set is not closed under R -> -R")
        out[i] = pos[key]
    return out


# ------------------------------------------------------------ electrons

def nn_hopping(R, t=-1.0):
    """Single-band nearest-neighbour hopping on the simple-cubic lattice:
    H(R) = t for the six vectors of length 1, 0 otherwise.  [N][1][1] c128."""
    R = np.asarray(R)
    H = np.zeros((len(R), 1, 1), dtype=np.complex128)
    H[np.sum(R * R, axis=1) == 1, 0, 0] = t
    return H


def random_hamiltonian(R, vectors, nb, seed, decay=1.5, scale=1.0):
    """Random Hermitian-symmetric H(R): complex normal entries times
    exp(-|R|/decay), symmetrised so that H(-R) = H(R)^dagger.  [N][nb][nb]."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((len(R), nb, nb, 2))
    Z = (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)
    m = _minus_index(R)
    H = 0.5 * (Z + np.conj(np.swapaxes(Z[m], 1, 2)))
    d = np.linalg.norm(cartesian(R, vectors), axis=1)
    return H * (scale * np.exp(-d / decay))[:, None, None]


# -------------------------------------------------------------- phonons

def spring_dynmat(R, vectors, atoms, shells, seed=None, k_const=1.0, scale=1.0):
    """Real-space dynamical matrix D(R) [N][3A][3A] (real, unit masses) of
    central springs between all atom pairs closer than the `shells`-th
    distinct interatomic distance.  Each bond (kappa in cell 0, kappa' in
    cell R) contributes -K b b^T to D(R)[kappa, kappa'] and +K b b^T to
    D(0)[kappa, kappa] (b the unit bond vector), so D is positive
    semidefinite and obeys the acoustic sum rule by construction.  K is
    k_const when seed is None, else U(0.5, 1.5) per bond (a bond and its
    reverse share K), drawn in bond enumeration order."""
    R = np.asarray(R)
    vectors = np.asarray(vectors, dtype=np.float64)
    atoms_c = np.asarray(atoms, dtype=np.float64)
    na = len(atoms_c)
    box = list(itertools.product(range(-3, 4), repeat=3))
    cand = []
    for ka in range(na):
        for kb in range(na):
            for n in box:
                b = atoms_c[kb] + np.asarray(n, dtype=np.float64) @ vectors - atoms_c[ka]
                d = float(np.linalg.norm(b))
                if d > 1e-9:
                    cand.append((round(d, 9), ka, kb, n, b))
    dists = sorted({c[0] for c in cand})
    cutoff = dists[shells - 1]
    pos = {tuple(int(x) for x in r): i for i, r in enumerate(R)}
    rng = None if seed is None else np.random.default_rng(seed)
    kval = {}
    D = np.zeros((len(R), 3 * na, 3 * na))
    for d, ka, kb, n, b in cand:
        if d > cutoff:
            continue
        key = (ka, kb, n)
        rev = (kb, ka, tuple(-x for x in n))
        if rev in kval:
            K = kval[rev]
        elif rng is None:
            K = k_const
        else:
            K = float(rng.uniform(0.5, 1.5))
        kval[key] = K
        if n not in pos:
            raise ValueError("bond vector outside the real-space vector set")
        bh = b / np.linalg.norm(b)
        bb = K * np.outer(bh, bh)
        D[pos[n], 3 * ka:3 * ka + 3, 3 * kb:3 * kb + 3] -= bb
        D[pos[(0, 0, 0)], 3 * ka:3 * ka + 3, 3 * ka:3 * ka + 3] += bb
    return D * scale


def einstein_dynmat(R, nm, omega_e):
    """D(R) = omega_e^2 I at R = 0 only: every mode at omega_e for every q."""
    R = np.asarray(R)
    D = np.zeros((len(R), nm, nm))
    D[np.all(R == 0, axis=1)] = omega_e ** 2 * np.eye(nm)
    return D


# --------------------------------------------------------------- vertex

def random_vertex(Re, Rp, vectors, nm, nb, seed, g0, decay=1.0, rows_per_block=None):
    """g(R_e,R_p) [Ne][Np][nm][nb][nb] c128 with modulus
    g0 exp(-(|R_e| + |R_p|)/decay) and a uniform random phase, the phases
    drawn in (R_e, R_p, mode, m, n) C order.  Drawn a block of R_e rows at a
    time (the same stream as one draw of the whole array), so the largest
    systems need no temporaries beyond the output."""
    rng = np.random.default_rng(seed)
    de = np.linalg.norm(cartesian(Re, vectors), axis=1)
    dp = np.linalg.norm(cartesian(Rp, vectors), axis=1)
    out = np.empty((len(Re), len(Rp), nm, nb, nb), dtype=np.complex128)
    per_row = len(Rp) * nm * nb * nb
    step = rows_per_block or max(1, (1 << 24) // max(per_row, 1))
    for e0 in range(0, len(Re), step):
        e1 = min(len(Re), e0 + step)
        phi = 2.0 * np.pi * rng.random((e1 - e0, len(Rp), nm, nb, nb))
        mod = g0 * np.exp(-(de[e0:e1, None] + dp[None, :]) / decay)
        out[e0:e1] = mod[:, :, None, None, None] * np.exp(1j * phi)
    return out


def random_vertex_device(Re, Rp, vectors, nm, nb, seed, g0, decay=1.0, device="cuda"):
    """The distribution of random_vertex (same modulus, uniform phase), drawn
    on a device with torch's seeded generator: a different random stream,
    for throughput runs at sizes where host generation would dominate
    (617^2 x 9 x 16^2 entries).  Returns a complex128 device tensor."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    de = torch.as_tensor(np.linalg.norm(cartesian(Re, vectors), axis=1), device=device)
    dp = torch.as_tensor(np.linalg.norm(cartesian(Rp, vectors), axis=1), device=device)
    mod = g0 * torch.exp(-(de[:, None] + dp[None, :]) / decay)
    phi = torch.rand((len(Re), len(Rp), nm, nb, nb), generator=gen, device=device, dtype=torch.float64)
    phi.mul_(2.0 * np.pi)
    return torch.polar(mod[:, :, None, None, None].expand_as(phi).contiguous(), phi)


def constant_vertex(Re, Rp, c):
    """g_a(R_e,R_p) = c_a at R_e = R_p = 0 only (single band):
    the constant-coupling model of the closed-form linewidth."""
    Re = np.asarray(Re)
    Rp = np.asarray(Rp)
    c = np.asarray(c, dtype=np.complex128)
    g = np.zeros((len(Re), len(Rp), len(c), 1, 1), dtype=np.complex128)
    ie = int(np.flatnonzero(np.all(Re == 0, axis=1))[0])
    ip = int(np.flatnonzero(np.all(Rp == 0, axis=1))[0])
    g[ie, ip, :, 0, 0] = c
    return g


# --------------------------------------------------------------- points

def random_points(n, seed):
    """n uniform fractional points in [0,1)^3 (Sec. 10.1-10.2 random sets)."""
    return np.random.default_rng(seed).random((n, 3))


def loss_weights(nk, nb, seed):
    """w_nk ~ U(0,1) for the loss L = sum w Im Sigma."""
    return np.random.default_rng(seed).random((nk, nb))


# -------------------------------------------------------------- configs

# Scale constants fixed once against the FP64 oracle (the model spectra
# need an eigensolve, which this module does not do);
# tests/test_inputs.py recomputes each one and checks it.
#   realistic fcc model: bandwidth 12 eV and max omega 65 meV on the 6^3
#   coarse grid, mu = (max eps_4 + min eps_5)/2 + 0.1 eV on the 20^3 grid.
#   mobility-scale fcc model (8^3 coarse grid): bandwidth 12 eV and max
#   omega 65 meV on the coarse grid, band edges of bands 8 and 9 (1-based)
#   on the 40^3 grid, mu at their midpoint.
C5_H_SCALE = 0.16710290699251684
C5_D_SCALE = 0.0005428255495717735
C5_VBM = 0.8533556552525289
C5_CBM = -0.6980924543090177
C5_MU = 0.0776316004717556
C2_H_SCALE = 0.26863436263417284
C2_D_SCALE = 0.00038095141752211273
C2_MU = 0.020638396418062227


@dataclass
class Model:
    """Everything a run needs apart from the WS vector lists."""
    name: str
    metric: tuple
    vectors: np.ndarray
    coarse: tuple
    nb: int
    nm: int
    kgrid: tuple = None
    qgrid: tuple = None
    T: float = 300.0
    mu: float = 0.0
    sigma: float = 0.05
    omega_cut: float = 1e-3
    deg_tol: float = 1e-6
    extra: dict = field(default_factory=dict)


def toy_model(kgrid=(8, 8, 8), qgrid=(8, 8, 8)):
    """Simple-cubic, 1 atom, 1 band: t = -1 eV, NN springs with
    omega_max = 50 meV, coarse 4^3, T = 300 K, mu = 0, sigma = 50 meV."""
    return Model("toy", SC_METRIC, SC_VECTORS, (4, 4, 4), 1, 3, kgrid, qgrid,
                 T=300.0, mu=0.0, sigma=0.05, extra={"omega_max": 0.05, "seed_g": 0})


def toy_arrays(Re, Rp, model=None):
    """(HR, DR, gR) of the toy model on the given vector lists."""
    om = 0.05 if model is None else model.extra["omega_max"]
    HR = nn_hopping(Re, -1.0)
    DR = spring_dynmat(Rp, SC_VECTORS, ATOMS_SC1, shells=1, k_const=om * om / 4.0)
    gR = random_vertex(Re, Rp, SC_VECTORS, 3, 1, seed=0, g0=0.1, decay=1.0)
    return HR, DR, gR


def realistic_model():
    """fcc, 2 atoms, 8 bands, 6 modes, coarse 6^3, fine 20^3 x 20^3,
    T = 300 K, sigma = 20 meV, mu at mid-gap + 0.1 eV."""
    return Model("realistic", FCC_METRIC, FCC_VECTORS, (6, 6, 6), 8, 6,
                 (20, 20, 20), (20, 20, 20), T=300.0,
                 mu=C2_MU, sigma=0.02)


def polar_params(seed=30, z=2.0, eps=5.5, prefactor=0.5, alpha=10.0, cutoff=50.0):
    """Synthetic polar data for the two-atom fcc models (zincblende-like,
    atoms at ATOMS_FCC2, unit masses as the spring dynamical matrices): Born
    charges Z*_1 = z I + a random symmetric part (entries U(-0.2, 0.2)) and a
    random antisymmetric part (U(-0.1, 0.1)), Z*_2 = -Z*_1 (charge
    neutrality); eps_inf = eps I + a random symmetric part (U(-0.3, 0.3));
    the overall factor C, the Gaussian parameter alpha and the cutoff of the
    G sum."""
    rng = np.random.default_rng(seed)
    s = rng.uniform(-0.2, 0.2, (3, 3))
    a = rng.uniform(-0.1, 0.1, (3, 3))
    z1 = z * np.eye(3) + 0.5 * (s + s.T) + 0.5 * (a - a.T)
    e = rng.uniform(-0.3, 0.3, (3, 3))
    return {"vectors": FCC_VECTORS.copy(), "tau": ATOMS_FCC2.copy(), "zstar": np.stack([z1, -z1]),
            "eps_inf": eps * np.eye(3) + 0.5 * (e + e.T), "masses": np.ones(2), "prefactor": prefactor,
            "alpha": alpha, "cutoff": cutoff}


def line_points(a, b, n):
    """n fractional points from a to b inclusive (a band-structure path)."""
    t = np.linspace(0.0, 1.0, n)[:, None]
    return (1.0 - t) * np.asarray(a, dtype=np.float64)[None, :] + t * np.asarray(b, dtype=np.float64)[None, :]


def spectral_workload(nq=100000):
    """The frequency-resolved self-energy and spectral-function workload on
    the realistic system: 64 k points on the line Gamma -> X = (0, 1/2, 1/2)
    (two bands cross eps_F on it), nq uniform random q (seed 7; spectral
    functions are integrated on random q sets, Sec. 10.1), 512 frequencies on
    [-1, 1] eV from eps_F; T, mu and delta = sigma as the realistic model."""
    return {"k": line_points((0.0, 0.0, 0.0), (0.0, 0.5, 0.5), 64), "q": random_points(nq, 7),
            "wgrid": np.linspace(-1.0, 1.0, 512)}


def mobility_model():
    """The mobility-scale system: fcc, 3 atoms, 16 bands, 9 modes, coarse
    8^3 (617 WS vectors), 8000 k in a 0.3 eV window above the conduction
    band minimum, 125,000 random q in chunks of 4096, T = 300 K, sigma = 10 meV,
    mu at mid-gap (fixed at run time from the bands)."""
    return Model("mobility", FCC_METRIC, FCC_VECTORS, (8, 8, 8), 16, 9, None, None, T=300.0,
                 mu=0.0, sigma=0.01, extra={"nk": 8000, "nq": 125000, "chunk": 4096, "window": 0.3,
                                            "seed_h": 20, "seed_d": 21, "seed_g": 22,
                                            "seed_k": 3, "seed_q": 2, "bandwidth": 12.0,
                                            "omega_max": 0.065})


def mobility_unscaled(R):
    """(HR, DR) of the mobility-scale system before rescaling (seeds 20, 21;
    decay lengths as the realistic model)."""
    HR = random_hamiltonian(R, FCC_VECTORS, 16, seed=20, decay=1.5, scale=1.0)
    DR = spring_dynmat(R, FCC_VECTORS, ATOMS_FCC3, shells=2, seed=21, scale=1.0)
    return HR, DR


def mobility_arrays(R):
    """(HR, DR) of the mobility-scale system, rescaled by the constants above."""
    HR, DR = mobility_unscaled(R)
    return HR * C5_H_SCALE, DR * C5_D_SCALE


def mobility_vertex(R):
    """g(R_e,R_p) of the mobility-scale system on the host (seed 22; 14 GB at
    617 WS vectors)."""
    return random_vertex(R, R, FCC_VECTORS, 9, 16, seed=22, g0=0.05, decay=1.0)


def mobility_k_candidates(n, seed=3):
    """The uniform stream from which the 0.3 eV window keeps its k points."""
    return random_points(n, seed)


def realistic_arrays(Re, Rp, h_scale=None, d_scale=None):
    """(HR, DR, gR) of the realistic model (seeds 10, 11, 12)."""
    hs = C2_H_SCALE if h_scale is None else h_scale
    ds = C2_D_SCALE if d_scale is None else d_scale
    HR = random_hamiltonian(Re, FCC_VECTORS, 8, seed=10, decay=1.5, scale=hs)
    DR = spring_dynmat(Rp, FCC_VECTORS, ATOMS_FCC2, shells=2, seed=11, scale=ds)
    gR = random_vertex(Re, Rp, FCC_VECTORS, 6, 8, seed=12, g0=0.05, decay=1.0)
    return HR, DR, gR
