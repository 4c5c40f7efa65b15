"""Closed-form potential of a uniformly charged planar triangle, used only to
pin the singular (Sauter-Schwab) quadrature against an independent route.

    I(x) = int_T dy / |x - y|
         = sum_edges [ t0 ln((R+ + s+)/(R- + s-))
                       - |d| (atan(t0 s+ / (R0^2 + |d| R+)) - atan(t0 s- / (R0^2 + |d| R-))) ]

(classical result for polygonal sources, e.g. Wilton et al. 1984): d is the
height of x above the plane, t0 the signed in-plane distance of the projected
point to each edge line (positive inside), s-/s+ the edge-end abscissae along
the edge and R-/R+ the distances of x to the edge ends, R0^2 = t0^2 + d^2.

Outer integrals use a tanh-sinh rule on the collapsed square map of the
triangle, which resolves the logarithmic edge/vertex behaviour of I(x).
"""

from __future__ import annotations

import numpy as np


def triangle_potential(P: np.ndarray, x: np.ndarray) -> np.ndarray:
    """int_T 1/|x-y| dy for the triangle with vertex rows P (3,3), at points x (...,3)."""
    P = np.asarray(P, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    n = n / np.linalg.norm(n)
    d = np.einsum("...c,c->...", x - P[0], n)
    rho = x - d[..., None] * n
    ad = np.abs(d)
    out = np.zeros(x.shape[:-1])
    for i in range(3):
        A, B = P[i], P[(i + 1) % 3]
        lhat = (B - A) / np.linalg.norm(B - A)
        uhat = np.cross(lhat, n)                 # outward in-plane edge normal
        sm = np.einsum("...c,c->...", A - rho, lhat)
        sp = np.einsum("...c,c->...", B - rho, lhat)
        t0 = np.einsum("...c,c->...", A - rho, uhat)    # > 0 when rho is inside
        Rm = np.linalg.norm(x - A, axis=-1)
        Rp = np.linalg.norm(x - B, axis=-1)
        R02 = t0 * t0 + d * d
        with np.errstate(divide="ignore", invalid="ignore"):
            num = Rp + sp
            den = Rm + sm
            # numerically stable form when the projected point lies beyond the edge end
            logt = np.where((num > 1e-300) & (den > 1e-300), np.log(num / den),
                            np.log((Rm - sm) / np.maximum(Rp - sp, 1e-300)))
            term = np.where(np.abs(t0) > 0, t0 * logt, 0.0)
            at = np.arctan2(t0 * sp, R02 + ad * Rp) - np.arctan2(t0 * sm, R02 + ad * Rm)
        out += term - ad * at
    return out


def tanh_sinh(n: int, h: float | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Tanh-sinh nodes and weights on [0,1] with 2n+1 points."""
    if h is None:
        h = 3.2 / n
    t = h * np.arange(-n, n + 1)
    s = 0.5 * np.pi * np.sinh(t)
    x = 0.5 * (1.0 + np.tanh(s))
    # 1 - x without cancellation: e^{-s}/(e^{s}+e^{-s}) ... kept implicit via x
    w = h * 0.5 * (0.5 * np.pi * np.cosh(t)) / np.cosh(s) ** 2
    keep = (x > 0.0) & (x < 1.0) & (w > 0.0)
    return x[keep], w[keep]


def triangle_rule_tanh_sinh(P: np.ndarray, n: int = 60):
    """Points (M,3) and weights (M,) on triangle P via x = P0 + u(P1-P0) + u v (P2-P1)."""
    u, wu = tanh_sinh(n)
    U, Vv = np.meshgrid(u, u, indexing="ij")
    WU, WV = np.meshgrid(wu, wu, indexing="ij")
    area2 = np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    pts = P[0] + U[..., None] * (P[1] - P[0]) + (U * Vv)[..., None] * (P[2] - P[1])
    w = WU * WV * U * area2
    return pts.reshape(-1, 3), w.ravel()


def double_integral_inv_r(Pi: np.ndarray, Pj: np.ndarray, n: int = 60) -> float:
    """int_{T_i} int_{T_j} 1/|x-y| dy dx  via the closed-form inner integral."""
    x, w = triangle_rule_tanh_sinh(np.asarray(Pi, float), n)
    return float(np.sum(w * triangle_potential(Pj, x)))
