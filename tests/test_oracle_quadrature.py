"""Pins of the oracle's quadrature against exact integrals (CPU only)."""

import numpy as np
import pytest

from oracle import static
from oracle.quadrature import chi, gauss01, sauter_schwab, triangle_rule6


def _ref_monomial(a: int, b: int) -> float:
    """int over tau = {0 <= x2 <= x1 <= 1} of x1^a x2^b = 1/((b+1)(a+b+2))."""
    return 1.0 / ((b + 1) * (a + b + 2))


def test_rule6_is_degree4_exact_and_not_degree5():
    bary, w = triangle_rule6()
    # reference triangle with vertices (0,0), (1,0), (1,1): area 1/2
    P = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0]])
    x = bary @ P
    for a in range(5):
        for b in range(5 - a):
            val = 0.5 * np.sum(w * x[:, 0] ** a * x[:, 1] ** b)
            assert abs(val - _ref_monomial(a, b)) < 1e-15 * 10
    errs = [abs(0.5 * np.sum(w * x[:, 0] ** a * x[:, 1] ** (5 - a)) - _ref_monomial(a, 5 - a))
            for a in range(6)]
    assert max(errs) > 1e-6
    assert np.all(w > 0) and abs(w.sum() - 1.0) < 1e-15 and np.allclose(bary.sum(1), 1.0)


def test_gauss01_exact_degree():
    x, w = gauss01(5)
    for p in range(10):
        assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 1e-15
    assert abs(np.sum(w * x ** 10) - 1.0 / 11) > 1e-9


@pytest.mark.parametrize("kind", ["identical", "edge", "vertex"])
def test_sauter_schwab_integrates_polynomials_exactly(kind):
    """The transforms must tile tau x tau exactly once with the right Jacobian:
    separable monomials x^a y^b integrate to products of exact values."""
    xh, yh, w = sauter_schwab(kind, 6)
    rng = np.random.default_rng(1)
    for _ in range(12):
        a, b, c, d = rng.integers(0, 3, size=4)
        val = np.sum(w * xh[:, 0] ** a * xh[:, 1] ** b * yh[:, 0] ** c * yh[:, 1] ** d)
        ref = _ref_monomial(a, b) * _ref_monomial(c, d)
        assert abs(val - ref) < 1e-13 * ref


# A triangle, one sharing its edge P0-P1 and one sharing its vertex P0 (not coplanar).
_P = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.3, 0.9, 0.05]])
_Q = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.6, -0.7, 0.3]])
_R = np.array([[0.0, 0.0, 0.0], [-0.8, 0.2, 0.1], [-0.3, -0.6, -0.2]])


@pytest.mark.parametrize("kind,A,B", [("identical", _P, _P), ("edge", _P, _Q), ("vertex", _P, _R)])
def test_sauter_schwab_static_kernel_vs_closed_form(kind, A, B):
    """int int 1/|x-y| over touching triangles: Sauter-Schwab (n_G = 10) vs the
    closed-form inner potential with a tanh-sinh outer rule."""
    ref = static.double_integral_inv_r(A, B, 80)
    xh, yh, w = sauter_schwab(kind, 10)
    x = chi(A[0], A[1], A[2], xh)
    y = chi(B[0], B[1], B[2], yh)
    ja = np.linalg.norm(np.cross(A[1] - A[0], A[2] - A[0]))
    jb = np.linalg.norm(np.cross(B[1] - B[0], B[2] - B[0]))
    val = np.sum(w / np.linalg.norm(x - y, axis=1)) * ja * jb
    assert abs(val - ref) < 1e-10 * ref
    # and the default n_G = 5 is already accurate to ~1e-6
    xh, yh, w = sauter_schwab(kind, 5)
    val5 = np.sum(w / np.linalg.norm(chi(A[0], A[1], A[2], xh) - chi(B[0], B[1], B[2], yh), axis=1)) * ja * jb
    assert abs(val5 - ref) < 1e-5 * ref


def test_triangle_potential_far_point_vs_quadrature():
    pts, w = static.triangle_rule_tanh_sinh(_P, 80)
    for x in ([2.0, 1.5, 0.7], [0.3, 0.3, 0.2], [-1.0, 0.2, -0.4]):
        num = np.sum(w / np.linalg.norm(pts - np.array(x), axis=1))
        assert abs(static.triangle_potential(_P, np.array([x]))[0] - num) < 1e-11 * num
