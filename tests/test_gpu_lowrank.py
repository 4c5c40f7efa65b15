"""Low-rank covariance on the GPU (fosb_lowrank_*): the pivoted Cholesky
factor on the ladder's quadrature nodes, the per-level factors
Y_l = Z_l^{-1} Wgt_l L_l and the CT variance from them, against the oracle
(oracle/lowrank.py) on the plain workload's ladder (s = 1..3, k = 1):
* pivots and rank identical (integers, decided with the same tie rule);
* Sigma = Y_l1 Y_l2^H against the oracle's two-sided solve of the low-rank
  right-hand side, and the variance, to 1e-10 (FP64) / 1e-7 (mixed);
* the separable models (constant: rank 1; n(x).n(y): rank 3) equal the dense
  variance;
and at the mixed workload's full size (s = 2..5, N up to 30720, k = 5)
against the oracle's dense variance (tests/golden/mixed_k5_oracle.json)."""

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


@pytest.mark.parametrize("precision,tol_v", [("fp64", 1e-10), ("mixed", 1e-7)])
def test_lowrank_against_oracle(fz, oracle_levels, precision, tol_v):
    fosb, ctx, torch = fz
    from oracle import lowrank, uq
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    xh = workloads.angles_xz(61)
    lv = _levels(fosb, ctx, [workloads.icosphere(s) for s in (1, 2, 3)], 1.0, prec)
    cov = fosb.make_cov("gaussian", SIG, ELL)
    print(f"[gpu] low-rank {precision}: pivoted Cholesky on s=1..3 nodes, tol 1e-10", flush=True)
    lr = fosb.LowRank(ctx, lv, cov, 4000, 1e-10)
    olv = {s: oracle_levels(s) for s in (1, 2, 3)}
    X, N, off = lowrank.ladder_candidates(olv, 1, 3)
    piv, Lf, res = lowrank.pivoted_cholesky("gaussian", SIG, ELL, X, N, 4000, 1e-10)
    print(f"[gpu]   rank {lr.rank} (oracle {len(piv)}), residual {lr.residual:.2e} ({res:.2e})", flush=True)
    assert lr.rank == len(piv) and np.array_equal(lr.pivots, piv)
    assert abs(lr.residual - res) <= 1e-12   # remaining diagonal: sigma^2 minus a sum of squares, rounding ~1e-15
    Vo, blocks = lowrank.second_moment(olv, 1, 3, xh, Lf, off)
    var = lr.far_field_moments(1, 3, xh).cpu().numpy()
    ev = _rel(var, Vo)
    Y3, Y1 = lr.factor(2), lr.factor(0)
    S31 = (Y3 @ Y1.conj().T).cpu().numpy()
    es = _rel(S31, blocks[(3, 1)])
    Vd = uq.second_moment(None, 1.0, 1, 3, "gaussian", SIG, ELL, xh, levels=olv)[0]
    ed = _rel(var, Vd)
    print(f"[gpu]   variance vs oracle low-rank {ev:.2e}, Sigma(3,1) {es:.2e}, vs dense covariance {ed:.2e}",
          flush=True)
    assert ev < tol_v and es < max(tol_v, 1e-9) and ed < 1e-7
    lr.close()


@pytest.mark.parametrize("kind,rank", [("constant", 1), ("normal_dot", 3)])
def test_lowrank_separable_models(fz, oracle_levels, kind, rank):
    fosb, ctx, torch = fz
    from oracle import uq
    xh = workloads.angles_xz(37)
    lv = _levels(fosb, ctx, [workloads.icosphere(s) for s in (1, 2, 3)], 1.0, fosb.FP64)
    cov = fosb.make_cov(kind, SIG, ELL)
    lr = fosb.LowRank(ctx, lv, cov, 64, 1e-12)
    olv = {s: oracle_levels(s) for s in (1, 2, 3)}
    Vd = uq.second_moment(None, 1.0, 1, 3, kind, SIG, ELL, xh, levels=olv)[0]
    var = lr.far_field_moments(1, 3, xh).cpu().numpy()
    print(f"[gpu] low-rank {kind}: rank {lr.rank}, vs dense {_rel(var, Vd):.2e}", flush=True)
    assert lr.rank == rank and _rel(var, Vd) < 1e-10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-7), ("mixed", 1e-6)])
def test_lowrank_full_size(fz, precision, tol):
    """Mixed workload at full size with the low-rank covariance (tol 1e-11)
    against the oracle's dense CT variance."""
    fosb, ctx, torch = fz
    with open(os.path.join(HERE, "golden", "mixed_k5_oracle.json")) as f:
        gold = np.asarray(json.load(f)["variance"])
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    w = workloads.workload("mixed_k5")
    opts = fosb.opts_default(ir_tol=1e-8) if prec == fosb.MIXED else None
    lv = _levels(fosb, ctx, w.meshes, w.k, prec, opts)
    cov = fosb.make_cov(w.cov_kind, w.sigma, w.ell)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lr = fosb.LowRank(ctx, lv, cov, 4000, 1e-11)
    t1 = time.perf_counter()
    var = lr.far_field_moments(w.L0, w.L, w.angles).cpu().numpy()
    t2 = time.perf_counter()
    e = _rel(var, gold)
    print(f"[gpu] low-rank full size {precision}: rank {lr.rank}, residual {lr.residual:.1e}, factor {t1 - t0:.3f} s, "
          f"solves + far field {t2 - t1:.3f} s, vs oracle dense {e:.2e}", flush=True)
    assert e < tol
    lr.close()
