"""Dielectric scattering: the PMCHWT Galerkin system on RWG (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's DE problem (problem setting: the transmission problem with
relative permittivity eps_r and permeability mu_r inside, the multitrace
operators built from the EFIO T_k and the MFIO K_k, and the PMCHWT equation
(A_0 + A^_1) xi = f with the interior operator scaled by
eta = sqrt(mu_r / eps_r)).  Discretised here as the classic Galerkin PMCHWT
for the exterior total traces, written from the Stratton-Chu representation
(exterior medium: k0, eta0 = 1; interior: k1 = k0 sqrt(eps_r mu_r), eta):

  unknowns  J = n x H~ (H~ = eta0 H),  M = -n x E  on Gamma (outward n);
  the field radiated into medium i by (J, M) is
      E = eta_i E_ki J - H_ki M,      H~ = H_ki J + E_ki M / eta_i,
  with the paper's potentials E_k (electric) and H_k = curl int G (magnetic);
  the exterior field is E^inc + radiated_0(J, M) outside and zero inside,
  the interior field radiated_1(-J, -M) inside and zero outside.  Adding the
  tangential traces of the two extinction statements (their identity parts
  cancel, leaving principal values) and testing with every RWG function gives

      [ T0 + eta T1      K0 + K1          ] [J]   [e]
      [ -(K0 + K1)       T0 + T1 / eta    ] [M] = [h],

      T_i[m, n] = int int G_ki [-i k_i phi_m.phi_n + (i/k_i) div phi_m div phi_n]
                (the EFIE matrix of oracle.efie, = -int phi_m . E_ki phi_n),
      K_i[m, n] = int int phi_m(x) . (grad_x G_ki(x, y) x phi_n(y)) dx dy
                (principal value; the MFIO pairing),
      grad_x G_k = (i k R - 1) exp(i k R) / (4 pi R^3) (x - y),
      e[m] = int phi_m . E^inc,   h[m] = int phi_m . H~^inc,
      E^inc = p exp(i k0 d.x),    H~^inc = (d x p) exp(i k0 d.x).

The far field of the exterior scattered field E^sc = E_k0 J - H_k0 M
(E^sc ~ e^{ik0|x|} / (4 pi |x|) F):
      F(xh) = i k0 [ (I - xh xh^T) int J e^{-i k0 xh.y} - xh x int M e^{-i k0 xh.y} ].

Quadrature as for the EFIE: the 6-point rule on both triangles of
non-touching pairs, Sauter-Schwab on touching ones.  On identical flat
triangles the K integrand phi_m . ((x - y) x phi_n) vanishes (all three
vectors lie in the triangle's plane), so those blocks are zero.

The paper's validation of the DE second moment (sphere experiment) uses the
rank-one right-hand side M^2[f] = f (x) f, whose solution is xi (x) xi: on
the discrete level pairs C_l1l2 = b_l1 b_l2^H and Sigma_l1l2 = u_l1 u_l2^H,
and the combination-technique far-field "variance" approximates |F|^2.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import efie
from . import mesh as meshmod
from .quadrature import chi, sauter_schwab, touching_order
from .uq import ct_pairs


def grad_green(k: float, d: np.ndarray) -> np.ndarray:
    """grad_x G_k(x, y) for d = x - y (..., 3)."""
    R = np.sqrt(np.sum(d * d, axis=-1))
    g = (1j * k * R - 1.0) * np.exp(1j * k * R) / (4.0 * np.pi * R ** 3)
    return g[..., None] * d


def local_regular_k(m: meshmod.RWGMesh, k: float, I: np.ndarray, J: np.ndarray, bq=None) -> np.ndarray:
    """Local 3x3 MFIO blocks (P,3,3) of the triangle pairs (I[p], J[p]), 6-point rule on both:
      blk[a,b] = sum_pq w_p w_q phi_a(x_p) . (grad G(x_p, y_q) x phi_b(y_q))."""
    X, W, Phi, D = bq if bq is not None else efie.basis_at_points(m)
    d = X[I][:, :, None, :] - X[J][:, None, :, :]                  # (P,6,6,3)
    gG = grad_green(k, d) * (W[I][:, :, None] * W[J][:, None, :])[..., None]
    phj = np.swapaxes(Phi[J], 1, 2)                                 # (P,6 q,3 b,3)
    cr = np.cross(gG[:, :, :, None, :], phj[:, None, :, :, :])      # (P,6,6,3 b,3)
    return np.einsum("Papc,Ppqbc->Pab", Phi[I], cr)


def local_singular_k(m: meshmod.RWGMesh, k: float, kind: str, I: np.ndarray, J: np.ndarray,
                     n_gauss: int, batch: int = 64) -> np.ndarray:
    """Local 3x3 MFIO blocks of touching pairs of one kind with the Sauter-Schwab
    transforms (same integrand as local_regular_k); identical pairs are zero."""
    P = len(I)
    out = np.zeros((P, 3, 3), dtype=np.complex128)
    if kind == "identical":
        return out
    xh, yh, w = sauter_schwab(kind, n_gauss)
    a = np.arange(3)
    for b0 in range(0, P, batch):
        ii = np.asarray(I[b0:b0 + batch], dtype=np.int64)
        jj = np.asarray(J[b0:b0 + batch], dtype=np.int64)
        orders = [touching_order(m.F[i], m.F[j]) for i, j in zip(ii, jj)]
        Pi = m.V[np.array([o[0] for o in orders])]
        Pj = m.V[np.array([o[1] for o in orders])]
        x = chi(Pi[:, None, 0], Pi[:, None, 1], Pi[:, None, 2], xh[None])   # (B,M,3)
        y = chi(Pj[:, None, 0], Pj[:, None, 1], Pj[:, None, 2], yh[None])
        jac = (2.0 * m.area[ii]) * (2.0 * m.area[jj])
        gG = grad_green(k, x - y) * (w[None] * jac[:, None])[..., None]     # (B,M,3)
        phx = meshmod.rwg_eval(m, ii[:, None, None], a[None, :, None], x[:, None])   # (B,3,M,3)
        phy = meshmod.rwg_eval(m, jj[:, None, None], a[None, :, None], y[:, None])
        cr = np.cross(gG[:, None, :, :], phy)                                 # (B,3 b,M,3)
        out[b0:b0 + batch] = np.einsum("Bamc,Bbmc->Bab", phx, cr)
    return out


def assemble_k(m: meshmod.RWGMesh, k: float, n_gauss: int = 5) -> np.ndarray:
    """Dense MFIO matrix K (ne x ne): K = S Khat S^T over all ordered triangle
    pairs (6-point rule on non-touching pairs, Sauter-Schwab on touching ones).
    Small meshes: Khat (3 nt x 3 nt) is held whole."""
    nt = m.nt
    bq = efie.basis_at_points(m)
    I = np.repeat(np.arange(nt), nt)
    J = np.tile(np.arange(nt), nt)
    blk = np.zeros((nt * nt, 3, 3), dtype=np.complex128)
    tp = meshmod.touching_pairs(m)
    touch = np.zeros(nt * nt, dtype=bool)
    for pairs in tp.values():
        touch[pairs[:, 0] * nt + pairs[:, 1]] = True
    reg = np.nonzero(~touch)[0]
    for c0 in range(0, len(reg), 20000):
        ix = reg[c0:c0 + 20000]
        blk[ix] = local_regular_k(m, k, I[ix], J[ix], bq)
    for kind, pairs in tp.items():
        if len(pairs):
            blk[pairs[:, 0] * nt + pairs[:, 1]] = local_singular_k(m, k, kind, pairs[:, 0], pairs[:, 1], n_gauss)
    Khat = blk.reshape(nt, nt, 3, 3).transpose(0, 2, 1, 3).reshape(3 * nt, 3 * nt)
    S = efie.incidence(m)
    return np.asarray((S @ (S @ Khat.T).T))


def wavenumbers(k0: float, eps_r: float, mu_r: float):
    """(k1, eta): interior wavenumber and relative wave impedance."""
    return k0 * np.sqrt(eps_r * mu_r), np.sqrt(mu_r / eps_r)


def assemble(m: meshmod.RWGMesh, k0: float, eps_r: float, mu_r: float, n_gauss: int = 5) -> np.ndarray:
    """The 2N x 2N PMCHWT matrix (unknowns [J; M])."""
    k1, eta = wavenumbers(k0, eps_r, mu_r)
    T0 = efie.assemble(m, k0, n_gauss)
    T1 = efie.assemble(m, k1, n_gauss)
    K = assemble_k(m, k0, n_gauss) + assemble_k(m, k1, n_gauss)
    return np.block([[T0 + eta * T1, K], [-K, T0 + T1 / eta]])


def incident_rhs(m: meshmod.RWGMesh, k0: float, d: np.ndarray, pol: np.ndarray) -> np.ndarray:
    """[e; h] (2N): e[m] = int phi_m . p e^{i k0 d.x}, h[m] = int phi_m . (d x p) e^{i k0 d.x}
    (6-point rule)."""
    X, W, Phi, D = efie.basis_at_points(m)
    d = np.asarray(d, dtype=np.float64)
    pol = np.asarray(pol)
    ph = np.exp(1j * k0 * (X @ d)) * W                                   # (nt,6)
    S = efie.incidence(m)
    e = S @ np.einsum("tq,taqc,c->ta", ph, Phi, pol).ravel()
    h = S @ np.einsum("tq,taqc,c->ta", ph, Phi, np.cross(d, pol)).ravel()
    return np.concatenate([e, h])


def far_field_matrix(m: meshmod.RWGMesh, k0: float, xh: np.ndarray) -> np.ndarray:
    """FF (3, n_a, 2N): F_c(xh_i) = sum_m FF[c, i, m] [J; M]_m."""
    X, W, Phi, D = efie.basis_at_points(m)
    xh = np.asarray(xh, dtype=np.float64)
    ph = np.exp(-1j * k0 * np.einsum("ic,tqc->itq", xh, X)) * W[None]    # (n_a,nt,6)
    A = np.einsum("itq,taqc->itac", ph, Phi)                              # (n_a,nt,3 local,3 comp)
    proj = np.eye(3)[None] - xh[:, :, None] * xh[:, None, :]
    FJ = 1j * k0 * np.einsum("icd,itad->cita", proj, A)                   # (3,n_a,nt,3)
    FM = -1j * k0 * np.transpose(np.cross(xh[:, None, None, :], A), (3, 0, 1, 2))
    S = efie.incidence(m)
    n_a = xh.shape[0]
    fj = (FJ.reshape(3 * n_a, 3 * m.nt) @ S.T).reshape(3, n_a, m.ne)
    fm = (FM.reshape(3 * n_a, 3 * m.nt) @ S.T).reshape(3, n_a, m.ne)
    return np.concatenate([fj, fm], axis=2)


def solve(m: meshmod.RWGMesh, k0: float, eps_r: float, mu_r: float, d, pol, n_gauss: int = 5):
    """(Z, b, u): the PMCHWT matrix, right-hand side and solution [J; M]."""
    Z = assemble(m, k0, eps_r, mu_r, n_gauss)
    b = incident_rhs(m, k0, d, pol)
    return Z, b, np.linalg.solve(Z, b)


def far_field(m: meshmod.RWGMesh, k0: float, u: np.ndarray, xh: np.ndarray) -> np.ndarray:
    """Far field F (n_a, 3) of the traces u = [J; M]."""
    return np.einsum("cim,m->ic", far_field_matrix(m, k0, xh), u)


def rank_one_second_moment(meshes: dict[int, meshmod.RWGMesh], L0: int, L: int, k0: float, eps_r: float,
                           mu_r: float, d, pol, xh: np.ndarray, n_gauss: int = 5, systems=None):
    """The sphere experiment's rank-one DE second moment over the
    combination-technique index set: for every pair C = b_l1 b_l2^H, the
    two-sided solve Z_l1 Sigma Z_l2^H = C (LU of each level), and
        V[c, i] = sum_{Lambda_H} sign mult Re (FF_l1 Sigma FF_l2^H)[(c,i),(c,i)].
    systems (optional): {level: (Z, b)} already assembled.
    Returns (V (3, n_a), Sigma blocks by pair, per-level (Z, b, u))."""
    lev = {}
    for s in range(L0, L + 1):
        if systems is not None and s in systems:
            Z, b = systems[s][0], systems[s][1]
        else:
            Z = assemble(meshes[s], k0, eps_r, mu_r, n_gauss)
            b = incident_rhs(meshes[s], k0, d, pol)
        lu = sla.lu_factor(Z)
        lev[s] = (Z, b, sla.lu_solve(lu, b), lu, far_field_matrix(meshes[s], k0, xh))
    V = np.zeros((3, xh.shape[0]))
    blocks = {}
    for l1, l2, sgn, mult in ct_pairs(L0, L):
        C = np.outer(lev[l1][1], lev[l2][1].conj())
        Y = sla.lu_solve(lev[l1][3], C)
        Sig = sla.lu_solve(lev[l2][3], Y.conj().T).conj().T
        blocks[(l1, l2)] = Sig
        F1, F2 = lev[l1][4], lev[l2][4]
        V += sgn * mult * np.real(np.einsum("cim,mn,cin->ci", F1, Sig, F2.conj()))
    return V, blocks, {s: lev[s][:3] for s in lev}
