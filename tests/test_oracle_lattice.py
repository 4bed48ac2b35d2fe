"""Pins for the oracle's integer steps (WS set, grids, k+q map)."""
import itertools

import numpy as np
import pytest

from oracle import lattice
from paper_1604_03525_amd import inputs as I

CASES = [(I.SC_METRIC, (4, 4, 4), 125, 64),
         (I.FCC_METRIC, (6, 6, 6), 279, 216),
         (I.FCC_METRIC, (8, 8, 8), 617, 512),
         (I.SC_METRIC, (3, 2, 5), None, 30),
         (I.FCC_METRIC, (1, 1, 1), None, 1)]


@pytest.mark.parametrize("metric,ncell,count,vol", CASES)
def test_ws_sum_rule_and_symmetry(metric, ncell, count, vol):
    R, nd = lattice.ws_vectors(metric, ncell)
    if count is not None:
        assert len(R) == count
    # the weights 1/ndeg tile the supercell exactly once: sum = N1 N2 N3
    from fractions import Fraction
    assert sum(Fraction(1, int(d)) for d in nd) == vol
    # closed under R -> -R with equal degeneracy
    pos = {tuple(r): d for r, d in zip(R.tolist(), nd.tolist())}
    for r, d in pos.items():
        assert pos[tuple(-x for x in r)] == d
    # lexicographic order
    assert [tuple(r) for r in R.tolist()] == sorted(tuple(r) for r in R.tolist())


@pytest.mark.parametrize("metric,ncell", [(I.SC_METRIC, (4, 4, 4)), (I.FCC_METRIC, (3, 3, 3)),
                                          (I.SC_METRIC, (2, 3, 4))])
def test_ws_brute_force_wider_shells(metric, ncell):
    """Membership and degeneracy against a brute force over a wider shift
    range {-3..3}^3 and a wider candidate box: the {-2..2} range suffices."""
    G = np.array(metric)
    N = np.array(ncell)
    R, nd = lattice.ws_vectors(metric, ncell)
    got = {tuple(r): d for r, d in zip(R.tolist(), nd.tolist())}
    shifts = np.array(list(itertools.product(range(-3, 4), repeat=3))) * N
    cand = np.array(list(itertools.product(*[range(-3 * x, 3 * x + 1) for x in ncell])))
    want = {}
    for n in cand:
        diff = n[None, :] - shifts
        ds = np.einsum("ta,ab,tb->t", diff, G, diff)
        d0 = n @ G @ n
        if ds.min() >= d0:
            want[tuple(n.tolist())] = int(np.sum(ds == d0))
    assert got == want


def test_grid_points_exact():
    g = lattice.grid_points(3, 4, 5)
    assert g.shape == (60, 3)
    i = (2 * 4 + 3) * 5 + 4
    assert tuple(g[i]) == (2 / 3, 3 / 4, 4 / 5)
    assert np.all(g >= 0) and np.all(g < 1)


@pytest.mark.parametrize("kg,qg", [((4, 4, 4), (4, 4, 4)), ((6, 4, 2), (3, 2, 1)),
                                   ((5, 5, 5), (5, 5, 5))])
def test_kq_index_is_k_plus_q(kg, qg):
    kq = lattice.kq_index(kg, qg)
    k = lattice.grid_points(*kg)
    q = lattice.grid_points(*qg)
    s = k[:, None, :] + q[None, :, :]
    t = k[kq]
    # equal modulo reciprocal lattice vectors, checked on integer numerators
    diff = (s - t) * np.array(kg)
    assert np.allclose(diff, np.round(diff), atol=1e-9)
    assert np.all(np.round(diff) % np.array(kg) == 0)
    # for each q the map k -> k+q is a permutation of the k grid
    for j in range(kq.shape[1]):
        assert sorted(kq[:, j].tolist()) == list(range(kq.shape[0]))


def test_kq_index_rejects_incommensurate():
    with pytest.raises(ValueError):
        lattice.kq_index((4, 4, 4), (3, 4, 4))
