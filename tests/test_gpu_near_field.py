"""Second moment of the field's shape derivative at field points
(fosb_near_field_moments) and the near-field map, against the oracle
(oracle/efie.py near_field_matrix, oracle/uq.py near_field_moments) on the
plain workload (s = 1..3, k = 1, Gaussian radial covariance), 48 seeded
points on the sphere of radius 2 and 16 at radius 1.3."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

SIG, ELL = 0.01, 0.5


@pytest.fixture(scope="module")
def fz():
    import torch
    from paper_2308_01457_amd import fosb
    assert torch.cuda.is_available()
    return fosb, fosb.Context(0), torch


def _points():
    g = np.random.default_rng(21).standard_normal((64, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return np.concatenate([2.0 * g[:48], 1.3 * g[48:]])


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-7)])
def test_near_field_moments_against_oracle(fz, oracle_levels, precision, tol):
    fosb, ctx, torch = fz
    from oracle import efie, uq
    prec = fosb.FP64 if precision == "fp64" else fosb.MIXED
    P = _points()
    levels = []
    for s in (1, 2, 3):
        m = fosb.Mesh(ctx, *workloads.icosphere(s))
        levels.append(fosb.Level(ctx, m, 1.0, fosb.assemble(ctx, m, 1.0), prec))
    NFg = fosb.near_field_matrix(ctx, levels[0], P).cpu().numpy().reshape(3, len(P), -1)
    olv = {s: oracle_levels(s) for s in (1, 2, 3)}
    NFo = efie.near_field_matrix(olv[1].mesh, 1.0, P)
    e_nf = float(np.abs(NFg - NFo).max() / np.abs(NFo).max())
    cov = fosb.make_cov("gaussian", SIG, ELL)
    blocks = fosb.correlation(ctx, levels, 1, 3, cov)
    print(f"[gpu] near field {precision}: 64 points", flush=True)
    var, mean = fosb.near_field_moments(ctx, levels, 1, 3, blocks, P)
    var, mean = var.cpu().numpy(), mean.cpu().numpy()
    _, _, oblocks, _, _ = uq.second_moment(None, 1.0, 1, 3, "gaussian", SIG, ELL, workloads.angles_xz(3), levels=olv)
    Vo, Mo = uq.near_field_moments(olv, oblocks, 1, 3, P)
    e_v, e_m = _rel(var, Vo), _rel(mean, Mo)
    print(f"[gpu]   near-field map {e_nf:.2e}, variance {e_v:.2e}, mean field {e_m:.2e}", flush=True)
    assert e_nf < 1e-12 and e_v < tol and e_m < max(tol, 1e-10)
