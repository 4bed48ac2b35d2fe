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


if __name__ == "__main__":
    h, d, mu = realistic_constants()
    print("C2_H_SCALE = %r" % float(h))
    print("C2_D_SCALE = %r" % float(d))
    print("C2_MU = %r" % float(mu))
