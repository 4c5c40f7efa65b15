"""EFIE Galerkin matrix, incident right-hand side and far-field map (FP64).

Definitions (problem-setting section: electric potential, EFIO T_k = {gamma_D E_k},
EFIE T_k j = gamma_D^c E^inc, far-field expansion; Galerkin section: Z u = b):

  With the pairing <u, v>_x = int u . (n x v) and gamma_D U = U x n,
  <T_k phi_n, phi_m>_x = -int phi_m . E_k phi_n; writing out E_k and moving
  the gradient onto phi_m by parts on the closed surface gives

      Z[m, n] = int int G_k(x, y) [ -i k phi_m(x).phi_n(y)
                                    + (i/k) div phi_m(x) div phi_n(y) ] dx dy,
      G_k(x, y) = exp(i k |x-y|) / (4 pi |x-y|),

      b[m] = <gamma_D E^inc, phi_m>_x = -int E^inc . phi_m,
      E^inc(x) = p exp(i k d.x)   (plane wave of the experiments section).

  The scattered field is E^sc = -E_k j, whose far field (E^sc ~ e^{ik|x|}/(4 pi |x|) F)
  is   F(xh) = -i k (I - xh xh^T) int j(y) exp(-i k xh.y) dy.

Quadrature: the 6-point rule on both triangles of every non-touching pair;
Sauter-Schwab (n_G points per dimension) on identical / edge- / vertex-adjacent
pairs.  Assembly is the plain sum over triangle pairs of the local 3x3
contributions, scattered onto the RWG indices by the incidence matrix S
(Z = S Zhat S^T).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import mesh as meshmod
from .quadrature import chi, sauter_schwab, touching_order, triangle_points


def incidence(m: meshmod.RWGMesh) -> sp.csr_matrix:
    """S (ne x 3nt): S[edge(t,a), 3t+a] = 1 (the sign lives in the basis)."""
    nt = m.nt
    rows = m.tri_edge.ravel()
    cols = np.arange(3 * nt)
    return sp.csr_matrix((np.ones(3 * nt), (rows, cols)), shape=(m.ne, 3 * nt))


def basis_at_points(m: meshmod.RWGMesh):
    """Quadrature nodes X (nt,6,3), weights W (nt,6), RWG values
    Phi (nt,3,6,3) and divergences D (nt,3) at the 6-point nodes."""
    X, W = triangle_points(m.V, m.F, m.area)
    t = np.arange(m.nt)[:, None, None]
    a = np.arange(3)[None, :, None]
    Phi = meshmod.rwg_eval(m, np.broadcast_to(t, (m.nt, 3, 6)), np.broadcast_to(a, (m.nt, 3, 6)),
                           X[:, None, :, :])
    D = meshmod.rwg_div(m, np.arange(m.nt)[:, None], np.arange(3)[None, :])
    return X, W, Phi, D


def green(k: float, R: np.ndarray) -> np.ndarray:
    return np.exp(1j * k * R) / (4.0 * np.pi * R)


def local_regular(m: meshmod.RWGMesh, k: float, I: np.ndarray, J: np.ndarray, bq=None) -> np.ndarray:
    """Local 3x3 EFIE blocks (P,3,3) of the aligned triangle pairs (I[p], J[p])
    with the 6-point rule on both triangles:
      blk[a,b] = sum_pq w_p w_q G(x_p,y_q) [-ik phi_a(x_p).phi_b(y_q) + (i/k) div phi_a div phi_b]."""
    X, W, Phi, D = bq if bq is not None else basis_at_points(m)
    d = X[I][:, :, None, :] - X[J][:, None, :, :]          # (P,6,6,3)
    R = np.sqrt(np.sum(d * d, axis=-1))
    G = green(k, R) * W[I][:, :, None] * W[J][:, None, :]  # (P,6,6)
    vec = np.zeros((len(I), 3, 3), dtype=np.complex128)
    for c in range(3):                                      # sum over vector components
        vec += Phi[I][..., c] @ G @ np.swapaxes(Phi[J][..., c], 1, 2)
    sca = np.sum(G, axis=(1, 2))[:, None, None] * D[I][:, :, None] * D[J][:, None, :]
    return -1j * k * vec + (1j / k) * sca


def local_singular(m: meshmod.RWGMesh, k: float, kind: str, I: np.ndarray, J: np.ndarray,
                   n_gauss: int, batch: int = 64) -> np.ndarray:
    """Local 3x3 EFIE blocks (P,3,3) of touching pairs of one kind, integrated
    with the Sauter-Schwab transforms (same integrand as local_regular)."""
    xh, yh, w = sauter_schwab(kind, n_gauss)
    P = len(I)
    out = np.zeros((P, 3, 3), dtype=np.complex128)
    for b0 in range(0, P, batch):
        ii = np.asarray(I[b0:b0 + batch], dtype=np.int64)
        jj = np.asarray(J[b0:b0 + batch], dtype=np.int64)
        orders = [touching_order(m.F[i], m.F[j]) for i, j in zip(ii, jj)]
        Pi = m.V[np.array([o[0] for o in orders])]          # (B,3,3) vertices P0,P1,P2
        Pj = m.V[np.array([o[1] for o in orders])]
        x = chi(Pi[:, None, 0], Pi[:, None, 1], Pi[:, None, 2], xh[None])   # (B,M,3)
        y = chi(Pj[:, None, 0], Pj[:, None, 1], Pj[:, None, 2], yh[None])
        jac = (2.0 * m.area[ii]) * (2.0 * m.area[jj])
        R = np.linalg.norm(x - y, axis=-1)
        G = green(k, R) * w[None] * jac[:, None]             # (B,M)
        a = np.arange(3)
        phx = meshmod.rwg_eval(m, ii[:, None, None], a[None, :, None], x[:, None])  # (B,3,M,3)
        phy = meshmod.rwg_eval(m, jj[:, None, None], a[None, :, None], y[:, None])
        Bn, M = G.shape
        lhs = (phx * G[:, None, :, None]).reshape(Bn, 3, 3 * M)
        vec = lhs @ np.swapaxes(phy.reshape(Bn, 3, 3 * M), 1, 2)
        dx = meshmod.rwg_div(m, ii[:, None], a[None, :])
        dy = meshmod.rwg_div(m, jj[:, None], a[None, :])
        out[b0:b0 + batch] = -1j * k * vec + (1j / k) * G.sum(axis=1)[:, None, None] * dx[:, :, None] * dy[:, None, :]
    return out


def _pool_map(fn, items, workers):
    if workers <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    from concurrent.futures import ThreadPoolExecutor   # numpy kernels release the GIL
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


def assemble(m: meshmod.RWGMesh, k: float, n_gauss: int = 5, chunk: int | None = None,
             workers: int | None = None) -> np.ndarray:
    """Dense EFIE matrix Z (ne x ne, complex128): Z = S Zhat S^T where Zhat holds
    the local 3x3 block of every ordered triangle pair (6-point rule on
    non-touching pairs, Sauter-Schwab on touching ones)."""
    import os
    workers = workers or os.cpu_count() or 1
    nt = m.nt
    bq = basis_at_points(m)
    S = incidence(m)
    tp = meshmod.touching_pairs(m)
    touch = sp.csr_matrix((np.ones(sum(len(v) for v in tp.values())),
                           (np.concatenate([v[:, 0] for v in tp.values()]),
                            np.concatenate([v[:, 1] for v in tp.values()]))), shape=(nt, nt))
    sing = {}
    for kind, pairs in tp.items():
        if len(pairs):
            parts = np.array_split(np.arange(len(pairs)), max(1, min(workers * 4, len(pairs) // 64)))
            blks = _pool_map(lambda ix: local_singular(m, k, kind, pairs[ix, 0], pairs[ix, 1], n_gauss),
                             parts, workers)
            for ix, blk in zip(parts, blks):
                for (i, j), b in zip(pairs[ix], blk):
                    sing[(int(i), int(j))] = b
    if chunk is None:
        chunk = max(1, min(nt, 400_000 // nt + 1))
    ST = S.T.tocsr()

    def rows_block(i0):
        rows = np.arange(i0, min(nt, i0 + chunk))
        I = np.repeat(rows, nt)
        J = np.tile(np.arange(nt), len(rows))
        with np.errstate(divide="ignore", invalid="ignore"):  # touching pairs are replaced below
            blk = local_regular(m, k, I, J, bq).reshape(len(rows), nt, 3, 3)
        tmask = touch[rows].toarray().astype(bool)
        blk[tmask] = 0.0
        for r, i in enumerate(rows):
            for j in np.nonzero(tmask[r])[0]:
                blk[r, j] = sing[(int(i), int(j))]
        Zhat = blk.transpose(0, 2, 1, 3).reshape(3 * len(rows), 3 * nt)
        Srows = S[:, 3 * i0: 3 * (i0 + len(rows))]
        edges = np.unique(Srows.nonzero()[0])         # the only rows this chunk contributes to
        return edges, Srows[edges] @ (Zhat @ ST)

    Z = np.zeros((m.ne, m.ne), dtype=np.complex128)
    starts = list(range(0, nt, chunk))
    for g0 in range(0, len(starts), workers):
        for edges, part in _pool_map(rows_block, starts[g0:g0 + workers], workers):
            Z[edges] += part
    return Z


def entries(m: meshmod.RWGMesh, k: float, rows: np.ndarray, cols: np.ndarray, n_gauss: int = 5) -> np.ndarray:
    """Selected entries Z[rows[p], cols[p]] computed one by one from their
    definition (sum over the four triangle pairs of the two supports)."""
    bq = basis_at_points(m)
    out = np.zeros(len(rows), dtype=np.complex128)
    for p, (mm, nn) in enumerate(zip(rows, cols)):
        acc = 0.0 + 0.0j
        for s in range(2):
            i, a = m.edge_tri[mm, s], m.edge_loc[mm, s]
            for t in range(2):
                j, b = m.edge_tri[nn, t], m.edge_loc[nn, t]
                ns = len(set(m.F[i].tolist()) & set(m.F[j].tolist()))
                if ns == 0:
                    blk = local_regular(m, k, np.array([i]), np.array([j]), bq)[0]
                else:
                    kind = {3: "identical", 2: "edge", 1: "vertex"}[ns]
                    blk = local_singular(m, k, kind, np.array([i]), np.array([j]), n_gauss)[0]
                acc += blk[a, b]
        out[p] = acc
    return out


def incident_rhs(m: meshmod.RWGMesh, k: float, d: np.ndarray, pol: np.ndarray) -> np.ndarray:
    """b[m] = -int p exp(i k d.x) . phi_m(x) dx  (6-point rule)."""
    X, W, Phi, D = basis_at_points(m)
    Einc = np.exp(1j * k * (X @ np.asarray(d, dtype=np.float64)))[..., None] * np.asarray(pol)[None, None, :]
    bhat = -np.einsum("tq,tqc,taqc->ta", W, Einc, Phi)
    return incidence(m) @ bhat.ravel()


def far_field_matrix(m: meshmod.RWGMesh, k: float, xh: np.ndarray) -> np.ndarray:
    """FF (3, n_a, ne): F_c(xh_i) = sum_m FF[c, i, m] u_m for j = sum u_m phi_m."""
    X, W, Phi, D = basis_at_points(m)
    xh = np.asarray(xh, dtype=np.float64)
    ph = np.exp(-1j * k * np.einsum("ic,tqc->itq", xh, X)) * W[None]          # (n_a,nt,6)
    J = np.einsum("itq,taqc->itac", ph, Phi)                                    # (n_a,nt,3,3)
    proj = np.eye(3)[None] - xh[:, :, None] * xh[:, None, :]                    # (n_a,3,3)
    Jt = -1j * k * np.einsum("icd,itad->cita", proj, J)                         # (3,n_a,nt,3)
    S = incidence(m)
    n_a = xh.shape[0]
    return (Jt.reshape(3 * n_a, 3 * m.nt) @ S.T).reshape(3, n_a, m.ne)


def near_field_matrix(m: meshmod.RWGMesh, k: float, P: np.ndarray) -> np.ndarray:
    """NF (3, n_p, ne): the scattered field E^sc_c(P_p) = sum_m NF[c, p, m] u_m
    of the current j = sum u_m phi_m at field points P (n_p, 3) off the
    surface, E^sc = -E_k j with the electric potential
        E_k phi(x) = i k int G(x, y) phi(y) dy + (i/k) grad_x int G(x, y) div phi(y) dy
    (the form whose Galerkin pairing is the EFIE matrix above, and whose far
    zone gives far_field_matrix), 6-point rule on every triangle,
    grad_x G = (i k - 1/R) G (x - y)/R."""
    X, W, Phi, D = basis_at_points(m)
    P = np.asarray(P, dtype=np.float64)
    d = P[:, None, None, :] - X[None]                                   # (n_p, nt, 6, 3)
    R = np.sqrt(np.sum(d * d, axis=-1))
    G = green(k, R) * W[None]                                           # (n_p, nt, 6)
    gG = ((1j * k - 1.0 / R) * G / R)[..., None] * d                    # (n_p, nt, 6, 3)
    t1 = np.einsum("ptq,taqc->ptac", G, Phi)
    t2 = np.einsum("ptqc,ta->ptac", gG, D)
    E = -(1j * k * t1 + (1j / k) * t2)                                  # (n_p, nt, 3 local, 3 comp)
    n_p = P.shape[0]
    Et = np.transpose(E, (3, 0, 1, 2)).reshape(3 * n_p, 3 * m.nt)
    return (Et @ incidence(m).T).reshape(3, n_p, m.ne)


def far_field(m: meshmod.RWGMesh, k: float, u: np.ndarray, xh: np.ndarray) -> np.ndarray:
    """Far field F (n_a, 3) of the current with RWG coefficients u."""
    FF = far_field_matrix(m, k, xh)
    return np.einsum("cim,m->ic", FF, u)
