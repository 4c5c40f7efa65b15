"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds geometry and draws parameters: closed triangle meshes
(vertices + outward-oriented triangles), incidence directions and polarisations,
observation directions and covariance parameters.  It holds none of the
boundary-element arithmetic (no basis functions, quadrature, kernels or
solves), so that the independent CPU oracle and the GPU library can both be fed
from it without sharing any of the method's code.

Meshes follow the paper's mesh hierarchy of planar triangulations with
h_l ~ q^{-l}, q = 2 (Galerkin section): level s of the icosphere has
20*4^s triangles and 30*4^s edges.  Triangles are emitted in subdivision
order (the four children of a parent are consecutive), which gives the
triangle and edge numbering spatial locality.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "icosahedron",
    "icosphere",
    "geodesic_sphere",
    "ellipsoid",
    "superquadric",
    "angles_xz",
    "kite_field",
    "kite_incidence",
    "Workload",
    "workload",
    "batched_ellipsoids",
]


def _orient_outward(V: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Flip every triangle whose normal points towards the origin (star-shaped
    closed surfaces around the origin only)."""
    P0, P1, P2 = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    nrm = np.cross(P1 - P0, P2 - P0)
    c = (P0 + P1 + P2) / 3.0
    flip = np.einsum("ij,ij->i", nrm, c) < 0
    F = F.copy()
    F[flip, 1], F[flip, 2] = F[flip, 2].copy(), F[flip, 1].copy()
    return F


def icosahedron() -> tuple[np.ndarray, np.ndarray]:
    """Regular icosahedron inscribed in the unit sphere, outward oriented."""
    phi = (1.0 + np.sqrt(5.0)) / 2.0
    pts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            pts.append((0.0, s1, s2 * phi))
            pts.append((s1, s2 * phi, 0.0))
            pts.append((s2 * phi, 0.0, s1))
    V = np.array(pts, dtype=np.float64)
    # faces = triples of mutually nearest-neighbour vertices (edge length 2)
    faces = []
    for a, b, c in itertools.combinations(range(12), 3):
        d = [np.linalg.norm(V[a] - V[b]), np.linalg.norm(V[b] - V[c]), np.linalg.norm(V[a] - V[c])]
        if all(abs(x - 2.0) < 1e-9 for x in d):
            faces.append((a, b, c))
    F = np.array(faces, dtype=np.int64)
    assert F.shape == (20, 3)
    V = V / np.linalg.norm(V, axis=1, keepdims=True)
    F = _orient_outward(V, F)
    return V, F.astype(np.int32)


def _subdivide(V: np.ndarray, F: np.ndarray, project) -> tuple[np.ndarray, np.ndarray]:
    verts = [tuple(v) for v in V]
    cache: dict[tuple[int, int], int] = {}

    def mid(a: int, b: int) -> int:
        key = (a, b) if a < b else (b, a)
        if key not in cache:
            m = 0.5 * (np.asarray(verts[a]) + np.asarray(verts[b]))
            cache[key] = len(verts)
            verts.append(tuple(project(m)))
        return cache[key]

    out = []
    for a, b, c in F:
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        out.extend([(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)])
    return np.array(verts, dtype=np.float64), np.array(out, dtype=np.int32)


def _unit(x: np.ndarray) -> np.ndarray:
    return x / np.linalg.norm(x)


def icosphere(s: int, radius: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Icosphere of subdivision level s: 20*4^s triangles, 30*4^s edges,
    10*4^s + 2 vertices on the sphere of the given radius."""
    V, F = icosahedron()
    for _ in range(s):
        V, F = _subdivide(V, F, _unit)
    return V * radius, F


def geodesic_sphere(nu: int) -> tuple[np.ndarray, np.ndarray]:
    """Frequency-nu geodesic sphere: every icosahedron face is split into a
    nu x nu barycentric grid (20*nu^2 triangles) projected to the unit sphere."""
    V0, F0 = icosahedron()
    key_to_id: dict[tuple, int] = {}
    verts: list[np.ndarray] = []
    tris: list[tuple[int, int, int]] = []

    def vid(face, i, j):
        a, b, c = face
        w = {a: nu - i - j, b: i, c: j}
        key = tuple(sorted((v, wt) for v, wt in w.items() if wt > 0))
        if key not in key_to_id:
            p = (w[a] * V0[a] + w[b] * V0[b] + w[c] * V0[c]) / nu
            key_to_id[key] = len(verts)
            verts.append(_unit(p))
        return key_to_id[key]

    for face in F0:
        for i in range(nu):
            for j in range(nu - i):
                tris.append((vid(face, i, j), vid(face, i + 1, j), vid(face, i, j + 1)))
                if i + j < nu - 1:
                    tris.append((vid(face, i + 1, j), vid(face, i + 1, j + 1), vid(face, i, j + 1)))
    V = np.array(verts, dtype=np.float64)
    F = np.array(tris, dtype=np.int32)
    return V, _orient_outward(V, F).astype(np.int32)


def ellipsoid(nu: int, axes: tuple[float, float, float]) -> tuple[np.ndarray, np.ndarray]:
    """Geodesic sphere scaled by axis-aligned semi-axes (a, b, c)."""
    V, F = geodesic_sphere(nu)
    return V * np.asarray(axes, dtype=np.float64)[None, :], F


def superquadric(s: int, p: float = 4.0) -> tuple[np.ndarray, np.ndarray]:
    """Closed surface |x|^p + |y|^p + |z|^p = 1, obtained by radially projecting
    the icosphere vertices: x = u / (sum |u_i|^p)^(1/p)."""
    V, F = icosphere(s)
    r = np.sum(np.abs(V) ** p, axis=1) ** (1.0 / p)
    return V / r[:, None], F


def angles_xz(n: int) -> np.ndarray:
    """n unit observation directions in the xz-plane, theta_i = pi*i/(n-1),
    x_hat = (sin theta, 0, cos theta)."""
    th = np.pi * np.arange(n) / (n - 1)
    return np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], axis=1)


def angles_xy(n: int) -> np.ndarray:
    """n unit observation directions in the plane z = 0, theta_i = 2 pi i / n
    (the angles of the experiments section), x_hat = (cos theta, sin theta, 0)."""
    th = 2.0 * np.pi * np.arange(n) / n
    return np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], axis=1)


def kite_field(X: np.ndarray) -> np.ndarray:
    """Deterministic perturbation field of the FOA-versus-ZOA experiment
    (kite experiment of the paper), evaluated at points X (..., 3):
    v(x) = ((z^2 - 1)(cos th - 1), 0.25 sin th (1 - z^2), 0), th = atan2(y, x)."""
    th = np.arctan2(X[..., 1], X[..., 0])
    z = X[..., 2]
    return np.stack([(z ** 2 - 1.0) * (np.cos(th) - 1.0), 0.25 * np.sin(th) * (1.0 - z ** 2), np.zeros_like(z)], -1)


def kite_incidence() -> tuple[np.ndarray, np.ndarray]:
    """Incidence (d, p) of the FOA-versus-ZOA experiment: d = (1, 2, 3)/sqrt(14)
    and the printed p = (i, 2, -1 - i/3) with its component along d removed
    (the printed vector has p.d != 0, which no plane wave satisfies)."""
    d = np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0)
    p = np.array([1j, 2.0, -1.0 - 1j / 3.0])
    return d, p - (p @ d) * d


def polarisation_for(d: np.ndarray) -> np.ndarray:
    """Real unit polarisation orthogonal to d: normalize(d x e_z), or e_x when
    d is (anti)parallel to e_z."""
    c = np.cross(d, np.array([0.0, 0.0, 1.0]))
    if np.linalg.norm(c) < 1e-6:
        return np.array([1.0, 0.0, 0.0])
    return c / np.linalg.norm(c)


@dataclass
class Workload:
    """One problem instance: a level ladder of meshes plus physical parameters."""

    name: str
    levels: list[int]                # level numbers s (icosphere subdivision counts)
    meshes: list[tuple[np.ndarray, np.ndarray]]
    k: float
    dirs: np.ndarray                 # (n_dirs, 3) incidence directions
    pols: np.ndarray                 # (n_dirs, 3) real polarisations
    cov_kind: str                    # "gaussian" | "matern32" | "constant" | "normal_dot"
    sigma: float
    ell: float
    L0: int
    L: int
    n_angles: int
    extra: dict = field(default_factory=dict)

    @property
    def angles(self) -> np.ndarray:
        return angles_xz(self.n_angles)


def workload(name: str, max_level: int | None = None) -> Workload:
    """The fixed (seed-free) single-shape workloads.

    plain_fp64  : unit icosphere s=1..3 (80/320/1280 triangles), k=1
    mixed_k5    : unit icosphere s=2..5 (up to 20480 triangles), k=5
    grad_k3     : unit icosphere s=1..4, k=3, 91 angles
    superquad_k8: superquadric |x|^4+|y|^4+|z|^4=1, s=3..6, k=8, 361 angles
    All use d=e_z, p=e_x and a radial Gaussian covariance.
    ``max_level`` truncates the ladder (tests at reduced size)."""
    ez = np.array([[0.0, 0.0, 1.0]])
    ex = np.array([[1.0, 0.0, 0.0]])
    if name == "plain_fp64":
        lv, mk, k, sig, ell, na = [1, 2, 3], icosphere, 1.0, 0.01, 0.5, 181
    elif name == "mixed_k5":
        lv, mk, k, sig, ell, na = [2, 3, 4, 5], icosphere, 5.0, 0.01, 0.5, 181
    elif name == "grad_k3":
        lv, mk, k, sig, ell, na = [1, 2, 3, 4], icosphere, 3.0, 0.01, 0.5, 91
    elif name == "superquad_k8":
        lv, mk, k, sig, ell, na = [3, 4, 5, 6], superquadric, 8.0, 0.005, 0.3, 361
    else:
        raise KeyError(name)
    if max_level is not None:
        lv = [s for s in lv if s <= max_level]
    meshes = [mk(s) for s in lv]
    return Workload(name, lv, meshes, k, ez, ex, "gaussian", sig, ell, lv[0], lv[-1], na)


def batched_ellipsoids(n_shapes: int = 64, n_dirs: int = 16, seed: int = 0) -> list[Workload]:
    """Seeded batch of ellipsoids: semi-axes ~ U[0.7,1.3], k ~ U[1,4],
    correlation length ~ U[0.3,0.8], top geodesic frequency nu ~ U{8..16};
    levels nu, nu//2, nu//4; n_dirs directions uniform on the sphere;
    Matern-3/2 radial covariance with amplitude 0.01.  Draw order per shape:
    axes(3), k, ell, nu, then the directions (3*n_dirs normals)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_shapes):
        axes = rng.uniform(0.7, 1.3, size=3)
        k = float(rng.uniform(1.0, 4.0))
        ell = float(rng.uniform(0.3, 0.8))
        nu = int(rng.integers(8, 17))
        g = rng.standard_normal((n_dirs, 3))
        dirs = g / np.linalg.norm(g, axis=1, keepdims=True)
        pols = np.stack([polarisation_for(d) for d in dirs])
        nus = [nu // 4, nu // 2, nu]
        meshes = [ellipsoid(n, tuple(axes)) for n in nus]
        out.append(Workload(f"ellipsoid{i}", [0, 1, 2], meshes, k, dirs, pols, "matern32",
                            0.01, ell, 0, 2, 181, extra={"axes": axes, "nu": nus}))
    return out
