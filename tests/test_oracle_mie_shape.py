"""The mesh-free spectral reference for the shape-derivative variance of the
PEC sphere (oracle/mie_shape.py), and the oracle's discretised variance
against it (CPU).

The reference is checked against facts that do not involve the
shape-derivative data: the plane wave's own series, the PEC boundary
condition, the Mie far field (for the exterior solver), the radius
derivative of the Mie series (breathing mode) and the exact translation
identity F_c = exp(i k (d - x).c) F.  The discretised variance of the
radial Gaussian perturbation (oracle/uq.py) must then converge to it at
second order in the mesh width, as the first moment does against Mie."""

import numpy as np
import pytest
from scipy.special import eval_legendre

import workloads
from oracle import mie, mie_shape as ms, uq


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_kappa_is_the_funk_hecke_expansion_of_the_gaussian():
    """kappa_n (closed form through modified spherical Bessel functions)
    equals 2 pi int K(t) P_n(t) dt by quadrature, and the Mercer series
    sum (2n+1)/(4 pi) kappa_n P_n(t) rebuilds sigma^2 exp(-(2-2t)/(2 ell^2))."""
    sig, ell = 0.7, 0.5
    kap = ms.gaussian_kappa(sig, ell, 40)
    t, w = np.polynomial.legendre.leggauss(200)
    K = sig ** 2 * np.exp(-(2.0 - 2.0 * t) / (2.0 * ell ** 2))
    kq = np.array([2.0 * np.pi * np.sum(w * K * eval_legendre(n, t)) for n in range(41)])
    assert np.abs(kap - kq).max() < 1e-13 * kap[0]
    tt = np.linspace(-1, 1, 17)
    series = sum((2 * n + 1) / (4 * np.pi) * kap[n] * eval_legendre(n, tt) for n in range(41))
    assert np.abs(series - sig ** 2 * np.exp(-(1.0 - tt) / ell ** 2)).max() < 1e-14


def test_mie_field_series():
    """The incident part of the series is e_x exp(i k z); the total field is
    normal on r = 1 (PEC); the radial derivative matches a central
    difference; the scattered part at large r has the far field of mie.py."""
    k = 2.0
    th = np.array([0.3, 1.1, 2.0, 2.9])
    ph = np.array([0.2, 1.3, -2.0, 0.7])
    xh = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    for r in (1.0, 1.7):
        Ei = ms.mie_fields(k, r, th, ph, part="incident")
        ref = np.zeros_like(Ei)
        ref[:, 0] = np.exp(1j * k * r * xh[:, 2])
        assert np.abs(Ei - ref).max() < 1e-13
        h = 1e-5
        fd = (ms.mie_fields(k, r + h, th, ph) - ms.mie_fields(k, r - h, th, ph)) / (2 * h)
        assert np.abs(fd - ms.mie_fields(k, r, th, ph, derivative=True)).max() < 1e-8
    E = ms.mie_fields(k, 1.0, th, ph)
    tang = E - np.sum(E * xh, -1)[:, None] * xh
    assert np.abs(tang).max() < 1e-14 * np.abs(E).max()
    Ff = mie.pec_far_field(k, 1.0, xh)
    errs = []
    for r in (4000.0, 8000.0):       # E ~ e^{ikr}/(4 pi r) (F + O(1/r))
        Es = ms.mie_fields(k, r, th, ph, part="scattered")
        errs.append(_rel(Es * 4 * np.pi * r / np.exp(1j * k * r), Ff))
    assert errs[1] < 5e-4 and 1.9 < errs[0] / errs[1] < 2.1, errs


@pytest.mark.parametrize("k", [1.0, 5.0])
def test_exterior_solver_reproduces_mie_far_field(k):
    """The vector-harmonic exterior solver, given the tangential trace of the
    Mie scattered field on r = 1, returns the Mie far field (poles included)."""
    xh = workloads.angles_xz(37)
    F = ms.scattered_far_field_from_trace(k, xh)
    assert _rel(F, mie.pec_far_field(k, 1.0, xh)) < 1e-11


@pytest.mark.parametrize("k", [1.0, 5.0])
def test_breathing_and_translation_modes(k):
    """v = 1 (radius change) gives dF/da of the exact series; v = c.x
    (rigid translation by c) gives i k (d - x).c F(x)."""
    xh = workloads.angles_xz(37)
    sd = ms.SphereShapeDerivative(k, 2)
    Fb = np.sqrt(4 * np.pi) * sd.far_field(0, 0, xh)
    assert _rel(Fb, mie.pec_far_field_radius_derivative(k, 1.0, xh)) < 1e-9
    c = np.array([0.3, -0.5, 0.8])
    coef = {0: c[2], 1: (-c[0] + 1j * c[1]) / np.sqrt(2), -1: (c[0] + 1j * c[1]) / np.sqrt(2)}
    Ft = np.sqrt(4 * np.pi / 3) * sum(coef[m] * sd.far_field(1, m, xh) for m in (-1, 0, 1))
    d = np.array([0.0, 0.0, 1.0])
    ref = 1j * k * ((d[None] - xh) @ c)[:, None] * mie.pec_far_field(k, 1.0, xh)
    assert _rel(Ft, ref) < 1e-10


def test_discretised_gaussian_variance_converges_to_the_spectral_reference(oracle_levels):
    """Full-tensor variance of the radial Gaussian perturbation (sigma = 1,
    ell = 0.5, k = 1) on icospheres s = 1, 2, 3 against the mesh-free value:
    the error falls about 4x per refinement (O(h^2)) to below 1%."""
    xh = workloads.angles_xz(37)
    Vr = ms.variance_gaussian(1.0, 1.0, 0.5, xh)
    errs = []
    for s in (1, 2, 3):
        lv = oracle_levels(s)
        C = uq.rhs_correlation(lv, lv, "gaussian", 1.0, 0.5)
        FF = uq.far_field_matrix(lv, xh)
        errs.append(_rel(uq.pair_variance(FF, uq.two_sided_solve(lv, lv, C), FF), Vr))
    assert errs[-1] < 1e-2 and errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_stored_spectral_values_and_the_mixed_workload_golden():
    """tests/golden/mie_shape_oracle.json holds what oracle/mie_shape.py
    computes (k = 1 recomputed here), and the oracle's CT variance of the
    mixed workload (s = 2..5, k = 5; tests/golden/mixed_k5_oracle.json) is
    within 0.2% of the mesh-free k = 5 value."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    with open(os.path.join(here, "mie_shape_oracle.json")) as f:
        ms_gold = json.load(f)
    xh = workloads.angles_xz(181)
    V1 = ms.variance_gaussian(1.0, ms_gold["sigma"], ms_gold["ell"], xh)
    assert np.abs(V1 - np.asarray(ms_gold["variance"]["1.0"])).max() < 1e-12 * np.abs(V1).max()
    with open(os.path.join(here, "mixed_k5_oracle.json")) as f:
        ct = np.asarray(json.load(f)["variance"])
    assert _rel(ct, np.asarray(ms_gold["variance"]["5.0"])) < 2e-3
