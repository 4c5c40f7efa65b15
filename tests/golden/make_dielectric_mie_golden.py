"""Writes tests/golden/dielectric_mie_k3.json from the oracle's dielectric Mie
series (oracle/mie.py) alone.

The sphere experiment's reference: the far field F of the unit dielectric
sphere (eps_r 2.1, mu_r 1, exterior wavenumber 3) for the plane wave
e_z exp(3 i x), at the 1801 angles theta_i = 2 pi i / 1801 of the plane z = 0;
stored as |F_c|^2 per component c (the quantity the rank-one second moment
approximates) and as F_z.  A second or two.

    python tests/golden/make_dielectric_mie_golden.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import mie  # noqa: E402

OUT = os.path.join(HERE, "dielectric_mie_k3.json")


def main():
    xh = workloads.angles_xy(1801)
    F = mie.dielectric_far_field_oriented(3.0, 1.0, 2.1, 1.0, (1.0, 0.0, 0.0), (0.0, 0.0, 1.0), xh)
    rec = {"k0": 3.0, "eps_r": 2.1, "mu_r": 1.0, "d": [1.0, 0.0, 0.0], "p": [0.0, 0.0, 1.0], "n_angles": 1801,
           "abs_F2": (np.abs(F.T) ** 2).tolist(), "Fz_re": F[:, 2].real.tolist(), "Fz_im": F[:, 2].imag.tolist()}
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
