"""Pins of the dielectric shape-derivative oracle (oracle/pmchwt_sd.py): the
quadratic interpolant through the 6-point nodes, the first-order far field
against the radius derivative of the dielectric Mie series (uniform normal
perturbation) and against finite differences of re-meshed PMCHWT solves
(a non-uniform radial field), and the second moment against the translation
identity.  Material and incidence of the paper's sphere experiment."""

import numpy as np
import pytest

import workloads
from oracle import efie, mie, pmchwt, pmchwt_sd
from oracle import mesh as meshmod
from oracle.quadrature import triangle_rule6

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

K0, EPS = 3.0, 2.1
D, P = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def levels():
    """Normal-field levels (nu = 1, so Wgt = W) on s = 1, 2."""
    return {s: pmchwt_sd.Level(*workloads.icosphere(s), K0, EPS, D, P, field_kind="normal") for s in (1, 2)}


def test_lagrange_basis_through_the_nodes():
    """ell_q(node p) = delta_pq, and the basis reproduces every quadratic."""
    bary, _ = triangle_rule6()
    Cinv = pmchwt_sd.lagrange6()
    E = pmchwt_sd._mono(bary[:, 1], bary[:, 2]) @ Cinv
    assert np.abs(E - np.eye(6)).max() < 1e-12
    rng = np.random.default_rng(3)
    c = rng.normal(size=6)
    f = lambda l1, l2: c[0] + c[1] * l1 + c[2] * l2 + c[3] * l1 * l1 + c[4] * l1 * l2 + c[5] * l2 * l2
    l = rng.random((50, 2)) * 0.5
    interp = (pmchwt_sd._mono(l[:, 0], l[:, 1]) @ Cinv) @ f(bary[:, 1], bary[:, 2])
    assert np.abs(interp - f(l[:, 0], l[:, 1])).max() < 1e-12


def _mie_radius_derivative(xh, h=1e-3):
    f = lambda a: mie.dielectric_far_field_oriented(K0, a, EPS, 1.0, D, P, xh)
    return (-f(1 + 2 * h) + 8 * f(1 + h) - 8 * f(1 - h) + f(1 - 2 * h)) / (12 * h)


def test_breathing_mode_converges_to_mie(levels):
    """v_n = 1: the first-order far field is the radius derivative of the Mie
    series; the FOSB value converges at second order (0.35, 0.085), and
    planted mistakes in the data (the H-equation's sign, its removal, a
    conjugation) leave it at O(1) on s = 1."""
    xh = workloads.angles_xy(37)
    dF = _mie_radius_derivative(xh)
    errs = {}
    for s, lv in levels.items():
        du = np.linalg.solve(lv.Z, lv.Wgt @ np.ones(lv.Wgt.shape[1]))
        errs[s] = _rel(pmchwt.far_field(lv.mesh, K0, du, xh), dF)
    print(f"breathing vs Mie: s=1 {errs[1]:.3e}, s=2 {errs[2]:.3e}")
    assert errs[2] < 0.1 and errs[1] / errs[2] > 3.5
    lv = levels[1]
    ne = lv.mesh.ne
    v = np.ones(lv.Wgt.shape[1])
    for name, W in (("flip r_H", np.vstack([lv.Wgt[:ne], -lv.Wgt[ne:]])),
                    ("drop r_H", np.vstack([lv.Wgt[:ne], 0 * lv.Wgt[ne:]])), ("conjugate", lv.Wgt.conj())):
        e = _rel(pmchwt.far_field(lv.mesh, K0, np.linalg.solve(lv.Z, W @ v), xh), dF)
        print(f"  planted {name}: {e:.3f}")
        assert e > 2.0 * errs[1]


def test_first_order_against_finite_differences(levels):
    """A non-uniform radial field v(x) x/|x| on s = 1: central differences of
    the far field of re-meshed PMCHWT solves (vertices moved by t v x/|x|)
    settle at second order in t, onto the FOSB first-order far field up to the
    h-floor (6% on s = 1, 1.8% on s = 2)."""
    lv = levels[1]
    m = lv.mesh
    V, F = workloads.icosphere(1)
    xh = workloads.angles_xy(37)
    e = np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0)
    vfun = lambda xhat: 1.0 + 0.5 * (xhat @ e) + 0.3 * xhat[..., 2] ** 2
    X, _, _, _ = efie.basis_at_points(m)
    Xh = X / np.linalg.norm(X, axis=-1, keepdims=True)
    vn = (vfun(Xh) * np.einsum("tqc,tc->tq", Xh, m.normal)).ravel()
    Fp = pmchwt.far_field(m, K0, np.linalg.solve(lv.Z, lv.Wgt @ vn), xh)
    Vh = V / np.linalg.norm(V, axis=1, keepdims=True)
    fds = []
    for t in (0.02, 0.01, 0.005):
        Fs = []
        for sg in (1.0, -1.0):
            mt = meshmod.build(V + sg * t * vfun(Vh)[:, None] * Vh, F)
            _, _, ut = pmchwt.solve(mt, K0, EPS, 1.0, D, P)
            Fs.append(pmchwt.far_field(mt, K0, ut, xh))
        fds.append((Fs[0] - Fs[1]) / (2 * t))
    steps = [_rel(fds[1], fds[0]) * np.linalg.norm(fds[0]) / np.linalg.norm(Fp),
             _rel(fds[2], fds[1]) * np.linalg.norm(fds[1]) / np.linalg.norm(Fp)]
    floor = _rel(fds[2], Fp)
    print(f"FD steps {steps[0]:.2e} {steps[1]:.2e} (rate {steps[0] / steps[1]:.2f}), FD vs FOSB {floor:.3e}")
    assert steps[0] / steps[1] > 3.5 and floor < 0.08


def test_second_moment_translation_identity(levels):
    """Rigid translation c ~ N(0, sigma^2 I): v_n = c.n, covariance
    sigma^2 n(x).n(y), and F_c moves by the factor exp(i k0 (d - x).c), so
    Var[F'_c] = sigma^2 k0^2 |d - x|^2 |F_c|^2 for any scatterer; the
    dielectric second moment converges to it at second order."""
    xh = workloads.angles_xy(37)
    sig = 0.01
    errs = {}
    for s, lv in levels.items():
        V, blocks = pmchwt_sd.second_moment({s: lv}, s, s, "normal_dot", sig, 1.0, xh)
        F = pmchwt.far_field(lv.mesh, K0, lv.u, xh)
        ref = sig ** 2 * K0 ** 2 * np.sum((D[None, :] - xh) ** 2, axis=1)[None, :] * np.abs(F.T) ** 2
        errs[s] = _rel(V, ref)
        S = blocks[(s, s)]
        assert np.abs(S - S.conj().T).max() < 1e-12 * np.abs(S).max()
    print(f"translation identity: s=1 {errs[1]:.3e}, s=2 {errs[2]:.3e}")
    assert errs[2] < 0.04 and errs[1] / errs[2] > 3.0
