"""Integer lattice bookkeeping for the interpolation (oracle side).

Test infrastructure only (see oracle/__init__.py).

The paper interpolates from coarse k/q grids through maximally localised
Wannier functions (Sec. 1, Sec. 8 step (iii)) but does not print the
real-space sums.  The reading adopted here is the standard one: the
real-space vectors are the lattice vectors inside the Wigner-Seitz cell of
the coarse-grid supercell, each weighted by 1/ndeg where ndeg counts the
supercell images at the same (minimal) distance.  Distances use the integer
metric G_ab = a_a . a_b (in units where the metric is integral), so every
comparison is exact.
"""
import itertools

import numpy as np


def ws_vectors(metric, ncell):
    """Wigner-Seitz vectors of the supercell ncell[0] x ncell[1] x ncell[2].

    A lattice vector n (integer coordinates) belongs to the set iff
    |n|_G^2 <= |n - T|_G^2 for every supercell vector T = (N1 t1, N2 t2, N3 t3)
    with t in {-2..2}^3; ndeg(n) is the number of such T (T = 0 included)
    that attain equality.  Candidates n run over [-2N_a, 2N_a] per axis.
    Order: lexicographic ascending in (n1, n2, n3).  All arithmetic is int64.

    Returns (R [N][3] int64, ndeg [N] int64).
    """
    G = np.asarray(metric, dtype=np.int64).reshape(3, 3)
    N = np.array([int(x) for x in ncell], dtype=np.int64)
    t = np.array(list(itertools.product(range(-2, 3), repeat=3)), dtype=np.int64)
    T = t * N[None, :]                                   # [125][3]
    axes = [np.arange(-2 * N[a], 2 * N[a] + 1, dtype=np.int64) for a in range(3)]
    n = np.array(list(itertools.product(*axes)), dtype=np.int64)   # C order
    d0 = np.einsum("ia,ab,ib->i", n, G, n)
    diff = n[:, None, :] - T[None, :, :]                 # [cand][125][3]
    d = np.einsum("ita,ab,itb->it", diff, G, diff)
    inside = np.all(d0[:, None] <= d, axis=1)
    ndeg = np.sum(d == d0[:, None], axis=1)
    return n[inside], ndeg[inside]


def grid_points(n1, n2, n3):
    """Gamma-centred homogeneous grid (Sec. 8 and the examples of Sec. 10):
    point i = (i1*N2 + i2)*N3 + i3 has fractional coordinates
    (i1/N1, i2/N2, i3/N3).  Returns [N1*N2*N3][3] float64."""
    out = np.empty((n1 * n2 * n3, 3), dtype=np.float64)
    i = 0
    for i1 in range(n1):
        for i2 in range(n2):
            for i3 in range(n3):
                out[i, 0] = i1 / n1
                out[i, 1] = i2 / n2
                out[i, 2] = i3 / n3
                i += 1
    return out


def kq_index(kgrid, qgrid):
    """Index of k+q (folded into [0,1)^3) in the k grid, for commensurate
    Gamma-centred grids (each k-grid dimension a multiple of the q-grid's).
    Point k_i + q_j has integer coordinates (i_a + j_a N^k_a/N^q_a) mod N^k_a.
    Returns [Nk][Nq] int64 with Nk, Nq the grid sizes in C order."""
    K = np.array([int(x) for x in kgrid], dtype=np.int64)
    Q = np.array([int(x) for x in qgrid], dtype=np.int64)
    if np.any(K % Q != 0):
        raise ValueError("q grid must divide the k grid")
    ratio = K // Q
    ik = np.arange(K.prod(), dtype=np.int64)
    iq = np.arange(Q.prod(), dtype=np.int64)
    i = np.stack([ik // (K[1] * K[2]), (ik // K[2]) % K[1], ik % K[2]], axis=1)
    j = np.stack([iq // (Q[1] * Q[2]), (iq // Q[2]) % Q[1], iq % Q[2]], axis=1)
    s = (i[:, None, :] + (j * ratio)[None, :, :]) % K   # [Nk][Nq][3]
    return (s[..., 0] * K[1] + s[..., 1]) * K[2] + s[..., 2]
