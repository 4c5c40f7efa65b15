"""GPU path vs the oracle on the superquadric |x|^4 + |y|^4 + |z|^4 = 1
(icosphere vertices projected radially), levels s = 1..3, k = 8, radial
Gaussian covariance (sigma 0.005, ell 0.3), L0 = 1, L = 3, 361 angles: the
large-ladder workload's geometry and parameters on the levels the oracle
finishes in seconds.  FP64 1e-10, mixed (bench tolerance) 1e-6."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

K8, SIG, ELL = 8.0, 0.005, 0.3


@pytest.fixture(scope="module")
def oracle_sq():
    from oracle import uq
    levels = {s: uq.make_level(*workloads.superquadric(s), K8) for s in (1, 2, 3)}
    xh = workloads.angles_xz(361)
    V = uq.second_moment(None, K8, 1, 3, "gaussian", SIG, ELL, xh, levels=levels)[0]
    return V, xh


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_superquadric_variance_matches_oracle(oracle_sq, precision, tol):
    import torch
    from paper_2308_01457_amd import fosb
    Vo, xh = oracle_sq
    ctx = fosb.Context(0)
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    meshes = [fosb.Mesh(ctx, *workloads.superquadric(s)) for s in (1, 2, 3)]
    print(f"[gpu] superquadric s=1..3 k=8 {precision}", flush=True)
    var, _, _ = fosb.second_moment(ctx, meshes, 1, 3, K8, prec, fosb.make_cov("gaussian", SIG, ELL), xh,
                                   opts=fosb.opts_default(ir_tol=1e-8 if prec == fosb.MIXED else 1e-10))
    e = float(np.linalg.norm(var.cpu().numpy() - Vo) / np.linalg.norm(Vo))
    print(f"[gpu]   variance vs oracle {e:.2e}", flush=True)
    assert e < tol
