"""Recompute the model scale constants held in paper_1604_03525_amd/inputs.py.

Calls only the FP64 oracle (and the input generators).  Run:
    python tests/golden/calibrate_models.py
and paste the printed values into inputs.py; tests/test_inputs.py checks that
they still agree with this computation.
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))

from oracle import lattice, interp                      # noqa: E402
from paper_1604_03525_amd import inputs as I            # noqa: E402


def realistic_constants():
    m = I.realistic_model()
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    HR, DR, _ = I.realistic_arrays(R, R, h_scale=1.0, d_scale=1.0)
    kc = lattice.grid_points(*m.coarse)
    eps, _ = interp.bands(HR, R, nd, kc)
    h_scale = 12.0 / (eps.max() - eps.min())
    om, _ = interp.phonons(DR, R, nd, kc)
    d_scale = (0.065 / om.max()) ** 2
    HR2, _, _ = I.realistic_arrays(R, R, h_scale=h_scale, d_scale=d_scale)
    kf = lattice.grid_points(*m.kgrid)
    ef, _ = interp.bands(HR2, R, nd, kf)
    mu = 0.5 * (ef[:, 3].max() + ef[:, 4].min()) + 0.1
    return h_scale, d_scale, mu


def mobility_constants():
    """Scales of the mobility-scale model (8^3 coarse grid): 12 eV bandwidth
    and 65 meV top phonon on the coarse grid; the band edges (the maximum of
    band n_b/2 and the minimum of band n_b/2 + 1, 1-based) on the 40^3 grid and
    mu at their midpoint (mid-gap; the random bands may overlap)."""
    m = I.mobility_model()
    R, nd = lattice.ws_vectors(m.metric, m.coarse)
    H0, D0 = I.mobility_unscaled(R)
    kc = lattice.grid_points(*m.coarse)
    eps, _ = interp.bands(H0, R, nd, kc)
    h_scale = m.extra["bandwidth"] / (eps.max() - eps.min())
    om, _ = interp.phonons(D0, R, nd, kc)
    d_scale = (m.extra["omega_max"] / om.max()) ** 2
    kf = lattice.grid_points(40, 40, 40)
    ef = np.concatenate([interp.bands(H0 * h_scale, R, nd, kf[i:i + 8000])[0] for i in range(0, len(kf), 8000)])
    nv = m.nb // 2
    vbm, cbm = ef[:, nv - 1].max(), ef[:, nv].min()
    return h_scale, d_scale, vbm, cbm, 0.5 * (vbm + cbm)


if __name__ == "__main__":
    h, d, mu = realistic_constants()
    print("C2_H_SCALE = %r" % float(h))
    print("C2_D_SCALE = %r" % float(d))
    print("C2_MU = %r" % float(mu))
    h, d, vbm, cbm, mu = mobility_constants()
    print("C5_H_SCALE = %r" % float(h))
    print("C5_D_SCALE = %r" % float(d))
    print("C5_VBM = %r" % float(vbm))
    print("C5_CBM = %r" % float(cbm))
    print("C5_MU = %r" % float(mu))
