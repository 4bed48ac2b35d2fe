"""The seeded input generators: structure of the models and the scale
constants that were fixed against the oracle."""
import numpy as np

from oracle import lattice
from paper_1604_03525_amd import inputs as I


def test_realistic_constants_reproduce():
    import importlib.util, os
    path = os.path.join(os.path.dirname(__file__), "golden", "calibrate_models.py")
    spec = importlib.util.spec_from_file_location("calibrate_models", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    h, d, mu = mod.realistic_constants()
    assert abs(h - I.C2_H_SCALE) < 1e-12 * h
    assert abs(d - I.C2_D_SCALE) < 1e-12 * d
    assert abs(mu - I.C2_MU) < 1e-12


def test_mobility_constants_reproduce():
    import importlib.util, os
    path = os.path.join(os.path.dirname(__file__), "golden", "calibrate_models.py")
    spec = importlib.util.spec_from_file_location("calibrate_models", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    h, d, vbm, cbm, mu = mod.mobility_constants()
    assert abs(h - I.C5_H_SCALE) < 1e-12 * h
    assert abs(d - I.C5_D_SCALE) < 1e-12 * d
    assert abs(vbm - I.C5_VBM) < 1e-12 and abs(cbm - I.C5_CBM) < 1e-12 and abs(mu - I.C5_MU) < 1e-12


def test_random_vertex_blocks_reproduce_one_draw():
    """The vertex drawn a block of R_e rows at a time is the one-draw array."""
    R, nd = lattice.ws_vectors(I.FCC_METRIC, (3, 3, 3))
    g = I.random_vertex(R, R, I.FCC_VECTORS, 9, 16, seed=22, g0=0.05, rows_per_block=5)
    assert np.array_equal(g, I.random_vertex(R, R, I.FCC_VECTORS, 9, 16, seed=22, g0=0.05))
    rng = np.random.default_rng(22)
    phi = 2.0 * np.pi * rng.random(g.shape)
    de = np.linalg.norm(I.cartesian(R, I.FCC_VECTORS), axis=1)
    mod = 0.05 * np.exp(-(de[:, None] + de[None, :]))
    assert np.array_equal(g, mod[:, :, None, None, None] * np.exp(1j * phi))


def test_model_symmetries():
    R, nd = lattice.ws_vectors(I.FCC_METRIC, (6, 6, 6))
    HR, DR, gR = I.realistic_arrays(R, R)
    assert HR.shape == (279, 8, 8) and DR.shape == (279, 6, 6) and gR.shape == (279, 279, 6, 8, 8)
    pos = {tuple(r): i for i, r in enumerate(R.tolist())}
    mi = np.array([pos[tuple(-x for x in r)] for r in R.tolist()])
    assert np.array_equal(HR[mi], np.conj(np.swapaxes(HR, 1, 2)))
    assert np.array_equal(DR[mi], np.swapaxes(DR, 1, 2))
    # acoustic sum rule: sum over cells and partner atoms vanishes
    asr = DR.reshape(len(R), 2, 3, 2, 3).sum(axis=(0, 3))
    assert np.max(np.abs(asr)) < 1e-15
    # vertex modulus law
    assert np.isclose(np.abs(gR[pos[(0, 0, 0)], pos[(0, 0, 0)]]).max(), 0.05)


def test_toy_model_arrays():
    R, nd = lattice.ws_vectors(I.SC_METRIC, (4, 4, 4))
    HR, DR, gR = I.toy_arrays(R, R)
    assert HR.shape == (125, 1, 1) and DR.shape == (125, 3, 3) and gR.shape == (125, 125, 3, 1, 1)
    assert np.count_nonzero(HR) == 6
    kappa = 0.05 ** 2 / 4
    i0 = int(np.flatnonzero(np.all(R == 0, axis=1))[0])
    assert np.allclose(DR[i0], 2 * kappa * np.eye(3))
    ix = int(np.flatnonzero(np.all(R == [1, 0, 0], axis=1))[0])
    assert np.allclose(DR[ix], np.diag([-kappa, 0, 0]))


def test_generators_are_deterministic():
    a = I.random_points(5, 2)
    b = I.random_points(5, 2)
    assert np.array_equal(a, b)
