"""RWG tables on a closed planar triangulation (Galerkin section: meshes of
planar triangles, div-conforming lowest-order Raviart-Thomas/RWG functions).

Conventions (shared by name, not by code, with the GPU library):
  * local edge a of triangle t is the edge opposite vertex F[t, a];
  * edges are numbered in first-visit order: scanning t = 0..nt-1 and
    a = 0, 1, 2, an edge gets the next id when first met;  the first triangle
    that meets it is T+ (the lower-indexed one), the other is T-;
  * RWG function of edge e with free vertices p+ (in T+) and p- (in T-):
        phi = +l/(2A+) (x - p+) on T+,   phi = -l/(2A-) (x - p-) on T-,
    div phi = +l/A+ on T+ and -l/A- on T-.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


class MeshError(ValueError):
    pass


@dataclass
class RWGMesh:
    V: np.ndarray          # (nv, 3) float64
    F: np.ndarray          # (nt, 3) int
    area: np.ndarray       # (nt,)
    normal: np.ndarray     # (nt, 3) unit outward normals
    tri_edge: np.ndarray   # (nt, 3) edge id of local edge a
    tri_sign: np.ndarray   # (nt, 3) +1 if t is T+ of that edge, -1 if T-
    edge_len: np.ndarray   # (ne,)
    edge_tri: np.ndarray   # (ne, 2) [T+, T-]
    edge_loc: np.ndarray   # (ne, 2) local index of the edge in T+, T-

    @property
    def nt(self) -> int:
        return self.F.shape[0]

    @property
    def ne(self) -> int:
        return self.edge_len.shape[0]


def build(V: np.ndarray, F: np.ndarray) -> RWGMesh:
    """Validate a closed, 2-manifold, consistently outward-oriented,
    non-degenerate triangulation and build its RWG tables."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    if V.ndim != 2 or V.shape[1] != 3 or F.ndim != 2 or F.shape[1] != 3:
        raise MeshError("V must be (nv,3) and F (nt,3)")
    if not np.all(np.isfinite(V)):
        raise MeshError("non-finite vertex coordinates")
    if F.size == 0 or F.min() < 0 or F.max() >= V.shape[0]:
        raise MeshError("triangle vertex index out of range")
    nt = F.shape[0]
    P0, P1, P2 = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    cr = np.cross(P1 - P0, P2 - P0)
    dbl = np.linalg.norm(cr, axis=1)
    scale = max(np.abs(V).max(), 1e-300)
    if np.any(dbl <= 1e-14 * scale * scale):
        raise MeshError("degenerate triangle")
    area = 0.5 * dbl
    normal = cr / dbl[:, None]

    first: dict[tuple[int, int], int] = {}
    tri_edge = np.zeros((nt, 3), dtype=np.int64)
    tri_sign = np.zeros((nt, 3), dtype=np.float64)
    e_tri: list[list[int]] = []
    e_loc: list[list[int]] = []
    e_dir: list[tuple[int, int]] = []
    for t in range(nt):
        for a in range(3):
            u, v = int(F[t, (a + 1) % 3]), int(F[t, (a + 2) % 3])
            if u == v:
                raise MeshError("repeated vertex in triangle")
            key = (u, v) if u < v else (v, u)
            if key not in first:
                first[key] = len(e_tri)
                e_tri.append([t, -1])
                e_loc.append([a, -1])
                e_dir.append((u, v))
                tri_edge[t, a] = first[key]
                tri_sign[t, a] = 1.0
            else:
                e = first[key]
                if e_tri[e][1] != -1:
                    raise MeshError("non-manifold edge (more than two triangles)")
                if e_dir[e] != (v, u):
                    raise MeshError("inconsistent orientation across an edge")
                e_tri[e][1] = t
                e_loc[e][1] = a
                tri_edge[t, a] = e
                tri_sign[t, a] = -1.0
    edge_tri = np.array(e_tri, dtype=np.int64)
    if np.any(edge_tri[:, 1] < 0):
        raise MeshError("open surface (edge with one triangle)")
    edge_loc = np.array(e_loc, dtype=np.int64)
    a_vert = np.array([d[0] for d in e_dir])
    b_vert = np.array([d[1] for d in e_dir])
    edge_len = np.linalg.norm(V[a_vert] - V[b_vert], axis=1)
    # outward orientation: the enclosed signed volume must be positive
    vol = np.sum(np.einsum("ij,ij->i", P0, np.cross(P1, P2))) / 6.0
    if vol <= 0:
        raise MeshError("triangles are oriented inward")
    return RWGMesh(V, F, area, normal, tri_edge, tri_sign, edge_len, edge_tri, edge_loc)


def touching_pairs(mesh: RWGMesh) -> dict[str, np.ndarray]:
    """Ordered triangle pairs (i, j) that share at least one vertex, split by
    the number of shared vertices: 'identical' (3), 'edge' (2), 'vertex' (1)."""
    nv = mesh.V.shape[0]
    v2t: list[list[int]] = [[] for _ in range(nv)]
    for t in range(mesh.nt):
        for v in mesh.F[t]:
            v2t[int(v)].append(t)
    out = {"identical": [], "edge": [], "vertex": []}
    for i in range(mesh.nt):
        nb = set()
        for v in mesh.F[i]:
            nb.update(v2t[int(v)])
        for j in sorted(nb):
            ns = len(set(mesh.F[i].tolist()) & set(mesh.F[j].tolist()))
            out[{3: "identical", 2: "edge", 1: "vertex"}[ns]].append((i, j))
    return {k: np.array(v, dtype=np.int64).reshape(-1, 2) for k, v in out.items()}


def rwg_eval(mesh: RWGMesh, t: int | np.ndarray, a: int | np.ndarray, x: np.ndarray) -> np.ndarray:
    """Value of the RWG function of local edge a of triangle t at points x
    (..., 3) lying on t, with the T+/T- sign included."""
    t = np.asarray(t)
    a = np.asarray(a)
    e = mesh.tri_edge[t, a]
    s = mesh.tri_sign[t, a]
    p = mesh.V[mesh.F[t, a]]
    c = s * mesh.edge_len[e] / (2.0 * mesh.area[t])
    return c[..., None] * (x - p)


def rwg_div(mesh: RWGMesh, t, a) -> np.ndarray:
    """Surface divergence of the RWG function of local edge a on triangle t."""
    t = np.asarray(t)
    a = np.asarray(a)
    e = mesh.tri_edge[t, a]
    return mesh.tri_sign[t, a] * mesh.edge_len[e] / mesh.area[t]
