"""Writes tests/golden/ellipsoids_oracle.json from the FP64 oracle alone.

Workload: two shapes of the batched ellipsoid workload (64 seeded ellipsoids,
seed 0, 16 incidences each; see workloads.batched_ellipsoids): shape 1
(top geodesic frequency 16: 5120 triangles, 7680 RWG) and shape 2 (frequency
8: 1280 triangles, 1920 RWG), each with its three-level ladder, wavenumber,
Matern-3/2 radial covariance (sigma 0.01, its own ell), its 16 incidences
and 181 angles in the xz-plane.  Stored per shape and incidence: the CT
far-field variance (3 x 181).  The oracle factors each level once and solves
the incidences one by one.  About twenty minutes on 8 cores.

    python tests/golden/make_ellipsoids_golden.py
"""

import json
import os
import sys
import time

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import efie, mesh as meshmod, uq  # noqa: E402

OUT = os.path.join(HERE, "ellipsoids_oracle.json")
SHAPES = (1, 2)


def main():
    batch = workloads.batched_ellipsoids(64, 16, seed=0)
    rec = {"workload": "ellipsoids", "seed": 0, "n_shapes_in_batch": 64, "n_dirs": 16, "n_angles": 181,
           "shapes": []}
    for si in SHAPES:
        w = batch[si]
        xh = w.angles
        t0 = time.time()
        base = {}
        for s, (V, F) in enumerate(w.meshes):
            m = meshmod.build(V, F)
            Z = efie.assemble(m, w.k)
            base[s] = (m, Z, sla.lu_factor(Z))
        print(f"shape {si}: nu={w.extra['nu']} k={w.k:.4f} ell={w.ell:.4f} levels {time.time() - t0:.0f} s",
              flush=True)
        var = []
        for d in range(len(w.dirs)):
            levels = {}
            for s, (m, Z, lu) in base.items():
                b = efie.incident_rhs(m, w.k, w.dirs[d], w.pols[d])
                u = sla.lu_solve(lu, b)
                Wgt, X, Nq = uq.rhs_weights(m, w.k, u, "radial")
                levels[s] = uq.Level(m, w.k, Z, lu, u, X, Nq, Wgt)
            V, _, _, _, _ = uq.second_moment(None, w.k, w.L0, w.L, w.cov_kind, w.sigma, w.ell, xh, levels=levels)
            var.append(V.tolist())
        print(f"shape {si}: 16 incidences {time.time() - t0:.0f} s", flush=True)
        rec["shapes"].append({"index": si, "nu": [int(x) for x in w.extra["nu"]], "k": w.k, "ell": w.ell,
                              "axes": np.asarray(w.extra["axes"]).tolist(), "variance": var})
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
