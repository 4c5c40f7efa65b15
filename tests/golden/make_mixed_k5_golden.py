"""Writes tests/golden/mixed_k5_oracle.json from the FP64 oracle alone.

Workload: unit icosphere s = 2..5 (480 / 1920 / 7680 / 30720 RWG), k = 5,
d = e_z, p = e_x, radial Gaussian covariance (sigma 0.01, ell 0.5),
combination technique L0 = 2, L = 5, 181 angles in the xz-plane: the
workload the benchmark times.  Stored per CT pair: the pair's far-field
variance contribution Re diag(FF1 Sigma FF2^H) (3 x 181), 48 sampled Sigma
entries and 48 sampled C entries (indices from numpy PCG64 seed 1234); per
level: 32 sampled first-moment coefficients and the first-moment far field
(3 x 181); and the CT variance.  Needs about 35 GB of host memory and an
hour on 8 cores (the s = 5 assembly and LU dominate).

    python tests/golden/make_mixed_k5_golden.py
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
from oracle import efie, uq  # noqa: E402

OUT = os.path.join(HERE, "mixed_k5_oracle.json")


def cplx(a):
    a = np.asarray(a)
    return {"re": a.real.tolist(), "im": a.imag.tolist()}


def main():
    w = workloads.workload("mixed_k5")
    xh = w.angles
    rng = np.random.Generator(np.random.PCG64(1234))
    levels = {}
    rec = {"workload": "mixed_k5", "levels": w.levels, "k": w.k, "cov": [w.cov_kind, w.sigma, w.ell],
           "L0": w.L0, "L": w.L, "n_angles": int(w.n_angles), "seed": 1234, "per_level": {}, "pairs": []}
    for s, (V, F) in zip(w.levels, w.meshes):
        t0 = time.time()
        lv = uq.make_level(V, F, w.k, w.dirs[0], w.pols[0])
        lv.Z = None                               # the LU factors are all that is needed below
        levels[s] = lv
        idx = rng.integers(0, lv.n, 32)
        Ff = efie.far_field(lv.mesh, w.k, lv.u, xh)
        rec["per_level"][str(s)] = {"n": int(lv.n), "u_idx": idx.tolist(), "u": cplx(lv.u[idx]),
                                    "far_field": cplx(Ff)}
        print(f"level s={s}: N={lv.n} {time.time() - t0:.0f} s", flush=True)
    V = np.zeros((3, w.n_angles))
    for l1, l2, sgn, mult in uq.ct_pairs(w.L0, w.L):
        t0 = time.time()
        a, b = levels[l1], levels[l2]
        C = uq.rhs_correlation(a, b, w.cov_kind, w.sigma, w.ell)
        ci = rng.integers(0, a.n, 48), rng.integers(0, b.n, 48)
        Csamp = C[ci]
        S = uq.two_sided_solve(a, b, C)
        del C
        si = rng.integers(0, a.n, 48), rng.integers(0, b.n, 48)
        Vp = uq.pair_variance(uq.far_field_matrix(a, xh), S, uq.far_field_matrix(b, xh))
        V += sgn * mult * Vp
        rec["pairs"].append({"l1": l1, "l2": l2, "sign": sgn, "mult": mult, "pair_variance": Vp.tolist(),
                             "C_idx": [ci[0].tolist(), ci[1].tolist()], "C": cplx(Csamp),
                             "Sigma_idx": [si[0].tolist(), si[1].tolist()], "Sigma": cplx(S[si])})
        del S
        print(f"pair ({l1},{l2}): {time.time() - t0:.0f} s", flush=True)
    rec["variance"] = V.tolist()
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
