"""Writes tests/golden/grad_k3_oracle.json from the FP64 oracle alone.

Workload: unit icosphere s = 1..4 (120 / 480 / 1920 / 7680 RWG), k = 3,
d = e_z, p = e_x, radial Gaussian covariance (sigma 0.01, ell 0.5),
combination technique L0 = 1, L = 4, 91 angles in the xz-plane: the
differentiated workload.  Stored: the CT variance (3 x 91), the summed
variance S = sum V and its gradient (dS/dsigma, dS/dell) from the oracle's
analytic adjoint (linearity of S in the covariance), and the same gradient
by central differences of the Sigma route (h = 1e-5 in ell) as a cross-check.
About ten minutes on 8 cores.

    python tests/golden/make_grad_k3_golden.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import uq  # noqa: E402

OUT = os.path.join(HERE, "grad_k3_oracle.json")


def main():
    w = workloads.workload("grad_k3")
    xh = w.angles
    levels = {}
    for s, (V, F) in zip(w.levels, w.meshes):
        t0 = time.time()
        levels[s] = uq.make_level(V, F, w.k, w.dirs[0], w.pols[0])
        print(f"level s={s}: N={levels[s].n} {time.time() - t0:.0f} s", flush=True)
    t0 = time.time()
    V, _, _, _, _ = uq.second_moment(None, w.k, w.L0, w.L, w.cov_kind, w.sigma, w.ell, xh, levels=levels)
    S, g = uq.summed_variance_and_gradient(levels, w.L0, w.L, w.cov_kind, w.sigma, w.ell, xh)
    h = 1e-5
    Sp, _ = uq.summed_variance_and_gradient(levels, w.L0, w.L, w.cov_kind, w.sigma, w.ell + h, xh)
    Sm, _ = uq.summed_variance_and_gradient(levels, w.L0, w.L, w.cov_kind, w.sigma, w.ell - h, xh)
    print(f"moments and gradient: {time.time() - t0:.0f} s", flush=True)
    rec = {"workload": "grad_k3", "levels": w.levels, "k": w.k, "cov": [w.cov_kind, w.sigma, w.ell],
           "L0": w.L0, "L": w.L, "n_angles": int(w.n_angles), "variance": V.tolist(),
           "S": float(S), "S_sigma_route": float(V.sum()), "dS_dsigma": float(g[0]), "dS_dell": float(g[1]),
           "dS_dell_central_difference": float((Sp - Sm) / (2 * h))}
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print("wrote", OUT, rec["S"], rec["dS_dsigma"], rec["dS_dell"], rec["dS_dell_central_difference"])


if __name__ == "__main__":
    main()
