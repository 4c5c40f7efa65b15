"""Brute-force Monte Carlo on tiny meshes against the first-order second
moment (CPU).

Every realisation of the radial perturbation re-meshes the sphere,
re-assembles and re-solves the EFIE (oracle/mc.py), so these tests pin the
shape-derivative right-hand side (oracle/uq.py: rhs_weights), the covariance
sampling and the first-order far field against an independent computation.
Antithetic pairs (+v, -v) cancel the odd orders in t exactly, so
  * the mean of F_t differs from F by O(t^2)  (FOA: E[F_t] = F + O(t^2));
  * the Monte Carlo second moment of (F_t - F)/t tends to that of F'[v] at
    second order in t, down to a floor set by the mesh width h (the mesh
    motion and the first-order map agree only up to O(h));
  * that floor shrinks as the mesh is refined.
The same draws feed both sides, so the sampling noise cancels.
"""

import numpy as np
import pytest

import workloads
from oracle import efie, mc, uq

K = 1.0
TS = (0.04, 0.02, 0.01, 0.005)


def _setup(oracle_levels, s, n_pairs=4, seed=7):
    V, F = workloads.icosphere(s)
    lv = oracle_levels(s)
    xi = np.random.default_rng(seed).standard_normal((n_pairs, len(V)))
    vr = mc.vertex_samples(V, "gaussian", 1.0, 0.5, xi)
    vr = np.concatenate([vr, -vr])                  # antithetic pairs
    xh = workloads.angles_xz(19)
    Fp = mc.first_order_far_field(lv, F, vr, xh)    # (M, 3, n_a)
    F0 = mc.far_field(V, F, K, xh).T                # (3, n_a)
    return V, F, vr, xh, Fp, F0


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def sweep_s1(oracle_levels):
    V, F, vr, xh, Fp, F0 = _setup(oracle_levels, 1)
    out = []
    for t in TS:
        Ft = mc.mc_far_fields(V, F, K, xh, vr, t)
        out.append((t, Ft))
    return F0, Fp, out


def test_mc_mean_is_second_order(sweep_s1):
    """E[F_t] - F = O(t^2): the error drops 4x per halving of t."""
    F0, _, out = sweep_s1
    errs = [_rel(np.mean(Ft, axis=0), F0) for _, Ft in out]
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.6 < r < 4.4 for r in ratios), (errs, ratios)
    assert errs[0] < 1e-2, errs


def test_mc_variance_converges_at_second_order_to_the_first_order_moment(sweep_s1):
    """Var[(F_t - F)/t] (Monte Carlo) minus the first-order second moment
    E|F'|^2 on the same draws: the t-dependent part shrinks 4x per halving of
    t, and the limit (Richardson extrapolation) is the h-floor, a few percent
    on the 80-triangle sphere."""
    F0, Fp, out = sweep_s1
    Vlin = np.mean(np.abs(Fp) ** 2, axis=0)
    Vmc = [np.mean(np.abs((Ft - F0[None]) / t) ** 2, axis=0) for t, Ft in out]
    steps = [_rel(Vmc[i], Vmc[i + 1]) for i in range(len(Vmc) - 1)]
    ratios = [steps[i] / steps[i + 1] for i in range(len(steps) - 1)]
    assert all(3.0 < r < 5.0 for r in ratios), (steps, ratios)
    floor = _rel((4.0 * Vmc[-1] - Vmc[-2]) / 3.0, Vlin)
    assert floor < 5e-2, floor
    # the per-realisation fields agree to first order in t, down to the same kind of floor
    lin = [_rel((Ft - F0[None]) / t, Fp) for t, Ft in out]
    assert lin[-1] < 4e-2 and lin[0] > lin[-1], lin


def test_mc_floor_shrinks_with_the_mesh(oracle_levels, sweep_s1):
    """The h-floor of the previous test on the 320-triangle sphere is several
    times smaller than on the 80-triangle one (a wrong sign or a dropped term
    in the shape-derivative data would leave an O(1) discrepancy instead)."""
    F0, Fp, out = sweep_s1
    Vlin1 = np.mean(np.abs(Fp) ** 2, axis=0)
    Vmc1 = [np.mean(np.abs((Ft - F0[None]) / t) ** 2, axis=0) for t, Ft in out[-2:]]
    floor1 = _rel((4.0 * Vmc1[1] - Vmc1[0]) / 3.0, Vlin1)
    V, F, vr, xh, Fp2, F02 = _setup(oracle_levels, 2)
    Vlin2 = np.mean(np.abs(Fp2) ** 2, axis=0)
    Vmc2 = [np.mean(np.abs((mc.mc_far_fields(V, F, K, xh, vr, t) - F02[None]) / t) ** 2, axis=0)
            for t in TS[-2:]]
    floor2 = _rel((4.0 * Vmc2[1] - Vmc2[0]) / 3.0, Vlin2)
    assert floor2 < 1.5e-2 and floor1 / floor2 > 2.5, (floor1, floor2)


def test_foa_versus_zoa_t_sweep():
    """Deterministic perturbation x -> x + t v(x) with the kite experiment's
    field v, applied to the 320-triangle sphere (its incidence, made
    transverse): the zeroth-order approximation F misses F_t by O(t), the
    first-order one F + t F'[v] by O(t^2), down to a small h-floor."""
    V, F = workloads.icosphere(2)
    d, p = workloads.kite_incidence()
    lv = uq.make_level(V, F, K, d, p, "normal")
    xh = workloads.angles_xz(37)
    F0 = efie.far_field(lv.mesh, K, lv.u, xh).T
    Fp = mc.first_order_far_field_vector(lv, workloads.kite_field, xh)
    zoa, foa = [], []
    for t in (0.2, 0.1, 0.05, 0.025):
        Ft = mc.far_field(V + t * workloads.kite_field(V), F, K, xh, d=d, pol=p).T
        zoa.append(_rel(F0, Ft))
        foa.append(_rel(F0 + t * Fp, Ft))
    rz = [zoa[i] / zoa[i + 1] for i in range(3)]
    rf = [foa[i] / foa[i + 1] for i in range(3)]
    assert all(1.8 < r < 2.1 for r in rz), (zoa, rz)
    assert rf[0] > 3.4 and rf[1] > 3.4 and rf[2] > 3.0, (foa, rf)
    assert foa[-1] < 1e-3 and foa[-1] < 0.05 * zoa[-1], (foa, zoa)
