"""Variance-only (adjoint) route, fosb_far_field_variance_adjoint: the CT
far-field variance from P_l = FF_l Z_l^{-1} Wgt_l (one adjoint solve with
3 n_a right-hand sides per level) and the covariance, with no Sigma block.

* Plain workload (s = 1..3, k = 1, 181 angles), Gaussian and Matern-3/2:
  against the oracle's Sigma-route variance and the GPU's own Sigma route,
  and the mean field against the oracle's first-moment far field.
* Mixed workload at full size (s = 2..5, N up to 30720, k = 5): against the
  oracle variance of tests/golden/mixed_k5_oracle.json."""

import json
import os
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
SIG, ELL = 0.01, 0.5


@pytest.fixture(scope="module")
def fz():
    import torch
    from paper_2308_01457_amd import fosb
    assert torch.cuda.is_available()
    return fosb, fosb.Context(0), torch


def _levels(fosb, ctx, ladder, k, precision, opts=None):
    out = []
    for V, F in ladder:
        m = fosb.Mesh(ctx, V, F)
        out.append(fosb.Level(ctx, m, k, fosb.assemble(ctx, m, k), precision, opts=opts))
    return out


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("precision,kind,tol", [("fp64", "gaussian", 1e-10), ("fp64", "matern32", 1e-10),
                                                ("mixed", "gaussian", 1e-7)])
def test_adjoint_route_plain_workload(fz, oracle_levels, precision, kind, tol):
    fosb, ctx, torch = fz
    from oracle import efie, uq
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    xh = workloads.angles_xz(181)
    cov = fosb.make_cov(kind, SIG, ELL)
    print(f"[gpu] variance-only route {precision} {kind} s=1..3", flush=True)
    lv = _levels(fosb, ctx, [workloads.icosphere(s) for s in (1, 2, 3)], 1.0, prec)
    va, mean = fosb.far_field_variance_adjoint(ctx, lv, 1, 3, cov, xh, with_mean=True)
    va, mean = va.cpu().numpy(), mean.cpu().numpy()
    blocks = fosb.correlation(ctx, lv, 1, 3, cov)
    vs = fosb.far_field_moments(ctx, lv, 1, 3, blocks, xh).cpu().numpy()
    olv = {s: oracle_levels(s) for s in (1, 2, 3)}
    Vo = uq.second_moment(None, 1.0, 1, 3, kind, SIG, ELL, xh, levels=olv)[0]
    Fo = efie.far_field(olv[3].mesh, 1.0, olv[3].u, xh).T
    e_o, e_s, e_m = _rel(va, Vo), _rel(va, vs), _rel(mean, Fo)
    print(f"[gpu]   vs oracle {e_o:.2e}, vs Sigma route {e_s:.2e}, mean field {e_m:.2e}", flush=True)
    assert e_o < tol and e_s < tol and e_m < max(tol, 1e-10)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_adjoint_route_full_size_against_golden(fz, precision, tol):
    fosb, ctx, torch = fz
    with open(os.path.join(HERE, "golden", "mixed_k5_oracle.json")) as f:
        gold = json.load(f)
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    w = workloads.workload("mixed_k5")
    cov = fosb.make_cov(w.cov_kind, w.sigma, w.ell)
    opts = fosb.opts_default(ir_tol=1e-8) if prec == fosb.MIXED else None
    print(f"[gpu] variance-only route at full size, {precision}", flush=True)
    lv = _levels(fosb, ctx, w.meshes, w.k, prec, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    va = fosb.far_field_variance_adjoint(ctx, lv, w.L0, w.L, cov, w.angles).cpu().numpy()
    t1 = time.perf_counter()
    e = _rel(va, np.asarray(gold["variance"]))
    print(f"[gpu]   vs oracle golden {e:.2e} ({t1 - t0:.3f} s for 181 angles)", flush=True)
    assert e < tol
