"""Writes tests/golden/mie_shape_oracle.json from the oracle's mesh-free
spectral reference (oracle/mie_shape.py) alone.

The far-field variance Var[F'_c](x) of the shape derivative of the PEC unit
sphere under the radial Gaussian perturbation (sigma 0.01, ell 0.5) for the
plane wave e_x exp(i k z), at the 181 angles of the xz-plane, for k = 1 (the
plain workload) and k = 5 (the mixed workload).  The discretised CT variance
of those workloads converges to these values as the mesh is refined.  A few
tens of seconds.

    python tests/golden/make_mie_shape_golden.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import mie_shape  # noqa: E402

OUT = os.path.join(HERE, "mie_shape_oracle.json")


def main():
    xh = workloads.angles_xz(181)
    rec = {"sigma": 0.01, "ell": 0.5, "n_angles": 181, "variance": {}}
    for k in (1.0, 5.0):
        rec["variance"][str(k)] = mie_shape.variance_gaussian(k, 0.01, 0.5, xh).tolist()
        print(f"k = {k}: done", flush=True)
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
