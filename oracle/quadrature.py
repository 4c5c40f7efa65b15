"""Quadrature rules.

* Regular triangle pairs: the symmetric 6-point, degree-4 rule on a triangle
  (Strang-Fix / Dunavant), nodes and weights taken from their closed form.
* Touching triangle pairs (identical, common edge, common vertex): the
  Sauter-Schwab regularising transforms of [0,1]^4 with a tensor Gauss-Legendre
  rule of n_G points per dimension (the workload's "Duffy on touching pairs").

Reference triangle: tau = {(x1, x2): 0 <= x2 <= x1 <= 1}, with vertices
(0,0), (1,0), (1,1) mapped to P0, P1, P2 by chi(x) = P0 + x1 (P1-P0) + x2 (P2-P1)
(|Jacobian| = 2 * area).  For the common-edge case both triangles put the
shared edge on P0-P1 (same physical order); for the common-vertex case the
shared vertex is P0 of both.
"""

from __future__ import annotations

import numpy as np


def triangle_rule6() -> tuple[np.ndarray, np.ndarray]:
    """Barycentric nodes (6, 3) and weights (6,) summing to 1 of the symmetric
    6-point degree-4 rule.  Two orbits (1-2b, b, b) with
    b = (8 - sqrt(10) +- sqrt(38 - 44 sqrt(2/5))) / 18 and weights
    (620 +- sqrt(213125 - 53320 sqrt(10))) / 3720 (per unit area)."""
    r10 = np.sqrt(10.0)
    root = np.sqrt(38.0 - 44.0 * np.sqrt(0.4))
    b1 = (8.0 - r10 + root) / 18.0
    b2 = (8.0 - r10 - root) / 18.0
    wr = np.sqrt(213125.0 - 53320.0 * r10)
    w1 = (620.0 + wr) / 3720.0
    w2 = (620.0 - wr) / 3720.0
    bary = []
    wts = []
    for b, w in ((b1, w1), (b2, w2)):
        a = 1.0 - 2.0 * b
        for perm in ((a, b, b), (b, a, b), (b, b, a)):
            bary.append(perm)
            wts.append(w)
    return np.array(bary), np.array(wts)


def triangle_points(V: np.ndarray, F: np.ndarray, area: np.ndarray):
    """Physical 6-point nodes (nt, 6, 3) and absolute weights (nt, 6)."""
    bary, w = triangle_rule6()
    P = V[F]  # (nt, 3, 3)
    X = np.einsum("qv,tvc->tqc", bary, P)
    W = area[:, None] * w[None, :]
    return X, W


def gauss01(n: int) -> tuple[np.ndarray, np.ndarray]:
    """n-point Gauss-Legendre rule on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _cube(n: int):
    x, w = gauss01(n)
    g = np.meshgrid(x, x, x, x, indexing="ij")
    ww = np.meshgrid(w, w, w, w, indexing="ij")
    xi, e1, e2, e3 = (a.ravel() for a in g)
    wc = ww[0].ravel() * ww[1].ravel() * ww[2].ravel() * ww[3].ravel()
    return xi, e1, e2, e3, wc


def sauter_schwab(kind: str, n: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Points xhat (M,2), yhat (M,2) and weights (M,) such that
    int_tau int_tau f(xhat, yhat) ~= sum_m w_m f(xhat_m, yhat_m), with the
    singular set of the given kind at the origin of the [0,1]^4 parameters
    (Sauter & Schwab, Boundary Element Methods, sec. 5.2)."""
    xi, e1, e2, e3, wc = _cube(n)
    X, Y, Wt = [], [], []

    def add(x1, x2, y1, y2, jac):
        X.append(np.stack([x1, x2], axis=1))
        Y.append(np.stack([y1, y2], axis=1))
        Wt.append(wc * jac)

    if kind == "identical":
        jac = xi ** 3 * e1 ** 2 * e2
        add(xi, xi * (1 - e1 + e1 * e2), xi * (1 - e1 * e2 * e3), xi * (1 - e1), jac)
        add(xi * (1 - e1 * e2 * e3), xi * (1 - e1), xi, xi * (1 - e1 + e1 * e2), jac)
        add(xi, xi * e1 * (1 - e2 + e2 * e3), xi * (1 - e1 * e2), xi * e1 * (1 - e2), jac)
        add(xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * (1 - e2 + e2 * e3), jac)
        add(xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * (1 - e2), jac)
        add(xi, xi * e1 * (1 - e2), xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), jac)
    elif kind == "edge":
        j1 = xi ** 3 * e1 ** 2
        j2 = xi ** 3 * e1 ** 2 * e2
        add(xi, xi * e1 * e3, xi * (1 - e1 * e2), xi * e1 * (1 - e2), j1)
        add(xi, xi * e1, xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), j2)
        add(xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * e2 * e3, j2)
        add(xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), xi, xi * e1, j2)
        add(xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * e2, j2)
    elif kind == "vertex":
        jac = xi ** 3 * e2
        add(xi, xi * e1, xi * e2, xi * e2 * e3, jac)
        add(xi * e2, xi * e2 * e3, xi, xi * e1, jac)
    else:
        raise ValueError(kind)
    return np.concatenate(X), np.concatenate(Y), np.concatenate(Wt)


def chi(P0: np.ndarray, P1: np.ndarray, P2: np.ndarray, xh: np.ndarray) -> np.ndarray:
    """Affine map of reference points xh (..., 2) to the triangle (P0, P1, P2)."""
    return P0 + xh[..., 0:1] * (P1 - P0) + xh[..., 1:2] * (P2 - P1)


def touching_order(Fi: np.ndarray, Fj: np.ndarray) -> tuple[list[int], list[int]]:
    """Vertex orders (P0, P1, P2) of triangles i and j for the Sauter-Schwab
    parameterisation.  Shared vertices first, taken in triangle i's cyclic
    order starting from Fi[0]; the remaining vertex/vertices of each triangle
    follow in that triangle's own cyclic order."""
    si = [int(v) for v in Fi]
    sj = [int(v) for v in Fj]
    shared = [v for v in si if v in sj]
    if len(shared) == 3:
        return si, list(si)
    if len(shared) == 2:
        a, b = shared
        oi = [v for v in si if v not in shared][0]
        oj = [v for v in sj if v not in shared][0]
        return [a, b, oi], [a, b, oj]
    if len(shared) == 1:
        a = shared[0]
        ki = si.index(a)
        kj = sj.index(a)
        return [a, si[(ki + 1) % 3], si[(ki + 2) % 3]], [a, sj[(kj + 1) % 3], sj[(kj + 2) % 3]]
    raise ValueError("triangles do not touch")
