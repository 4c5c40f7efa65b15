"""Brute-force Monte Carlo of the perturbed scattering problem on tiny meshes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The first-order approximation (FOA section of the paper) replaces the far
field of the perturbed scatterer Gamma_t = {x + t v(x)} by F + t F'[v], so
that
    E[F_t] = F + O(t^2)          (centred v: the first-order term has mean 0)
    Var[(F_t - F)/t] = Var[F'] + O(t)   in general, O(t^2) for antithetic
                                        (+v, -v) sample pairs,
and the combination technique computes Var[F'] = E|F'|^2 from the second
moment of v alone.  This module computes the left-hand sides by brute force:
every realisation re-meshes the scatterer, re-assembles and re-solves the
Galerkin EFIE, and takes the far field.  It is independent of the
shape-derivative machinery of uq.py (it never forms a shape-derivative
right-hand side) and so pins it.

Random field: v = v_r(x) x/|x| (radial perturbation).  Realisations of v_r
are drawn at the mesh vertices from N(0, K_vertices) (the caller passes the
standard-normal draws in; the Cholesky factor is formed here), each vertex x
moves to x + t v_r(x) x/|x|, and the same vertex values, interpolated
linearly over each flat triangle, feed the first-order map at the quadrature
nodes.  The two then describe the same random field up to the mesh width.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import efie
from . import mesh as meshmod
from . import uq
from .quadrature import triangle_rule6


def vertex_samples(V: np.ndarray, kind: str, sigma: float, ell: float, xi: np.ndarray) -> np.ndarray:
    """Realisations (M, nv) of v_r at the vertices: v = L xi with K = L L^T the
    covariance between vertices (Euclidean distance) and xi (M, nv) standard
    normal draws supplied by the caller."""
    K = uq.covariance(kind, sigma, ell, V, None, V, None)
    Lc = np.linalg.cholesky(K + 1e-12 * sigma ** 2 * np.eye(len(V)))
    return xi @ Lc.T


def perturbed_vertices(V: np.ndarray, vr: np.ndarray, t: float) -> np.ndarray:
    """x -> x + t v_r(x) x/|x| at every vertex."""
    return V + t * vr[:, None] * V / np.linalg.norm(V, axis=1, keepdims=True)


def far_field(V: np.ndarray, F: np.ndarray, k: float, xh: np.ndarray, d=(0.0, 0.0, 1.0),
              pol=(1.0, 0.0, 0.0), n_gauss: int = 5) -> np.ndarray:
    """Far field (n_a, 3) of the Galerkin EFIE solution on the mesh (V, F)."""
    m = meshmod.build(V, F)
    Z = efie.assemble(m, k, n_gauss=n_gauss)
    b = efie.incident_rhs(m, k, np.asarray(d, float), np.asarray(pol))
    u = sla.lu_solve(sla.lu_factor(Z), b)
    return efie.far_field(m, k, u, xh)


def vertex_to_nodes(F: np.ndarray, vr: np.ndarray) -> np.ndarray:
    """Linear interpolation of vertex values vr (M, nv) to the 6 quadrature
    nodes of every triangle, in the (t, q) order of the RHS weights: (M, 6 nt)."""
    bary, _ = triangle_rule6()                       # (6, 3)
    vals = vr[:, F]                                   # (M, nt, 3)
    return np.einsum("mtv,qv->mtq", vals, bary).reshape(vr.shape[0], -1)


def first_order_far_field(level: uq.Level, F: np.ndarray, vr: np.ndarray, xh: np.ndarray) -> np.ndarray:
    """F'[v] (M, 3, n_a) of each realisation through the first-order map:
    b' = Wgt v_r(nodes), Z dj' = b', F' = FF dj'."""
    vq = vertex_to_nodes(F, vr)                       # (M, Q)
    bp = np.asarray(level.Wgt @ vq.T)                 # (N, M)
    dj = sla.lu_solve(level.lu, bp)
    FF = uq.far_field_matrix(level, xh)               # (3, n_a, N)
    return np.einsum("cim,mk->kci", FF, dj)


def first_order_far_field_vector(level: uq.Level, vfield, xh: np.ndarray) -> np.ndarray:
    """F'[v] (3, n_a) for a deterministic vector perturbation field v (a
    function of points (..., 3)): its normal component v.n at the quadrature
    nodes feeds the first-order map of a level built with field_kind
    'normal'."""
    vn = np.sum(vfield(level.X) * level.Nq, axis=-1)
    dj = sla.lu_solve(level.lu, level.Wgt @ vn)
    return np.einsum("cim,m->ci", uq.far_field_matrix(level, xh), dj)


def mc_far_fields(V: np.ndarray, F: np.ndarray, k: float, xh: np.ndarray, vr: np.ndarray, t: float,
                  n_gauss: int = 5, workers: int = 1) -> np.ndarray:
    """Far fields (M, 3, n_a) of the meshes perturbed by t vr[j] for each
    realisation j (one assembly and solve per realisation)."""
    def one(j):
        return far_field(perturbed_vertices(V, vr[j], t), F, k, xh, n_gauss=n_gauss).T
    if workers <= 1:
        return np.stack([one(j) for j in range(vr.shape[0])])
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return np.stack(list(ex.map(one, range(vr.shape[0]))))
