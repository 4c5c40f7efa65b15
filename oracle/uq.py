"""Second moment of the shape derivative: right-hand side, tensor solves,
combination technique and far-field variance (FP64).

Definitions followed (FOA section, Galerkin section, combination-technique
subsection of the paper):

* Shape-derivative data.  For a realisation v_n of the normal velocity the
  shape derivative's trace solves T_k dj' = grad_G(v_n E_n) x n - i k v_n gamma_T H.
  With H = curl E/(ik) on the PEC surface, gamma_T H = n x j and
  E_n = (i/k) div_G j, so the Galerkin right-hand side is
      b'_m = int v_n [ (i/k) div j div phi_m - i k j . phi_m ].
  (The paper's four-term expansion of E[g (x) conj g] is garbled in print; the
  second moment is computed directly as C = E[b' b'^H].)
* Random field.  v_n(x) = v_r(x) nu(x): a scalar centred field v_r with
  covariance K, times nu = (x/|x|) . n (radial perturbation) or nu = 1 (the
  field is the normal velocity itself).  With quadrature weights folded in,
      b'_m = sum_q Wgt[m, q] v_r(x_q),    C = Wgt K Wgt^H.
* Tensor equation  (Z1 (x) conj Z2) vec Sigma = vec C, i.e. Z1 Sigma Z2^H = C,
  solved as Sigma = Z1^{-1} C Z2^{-H} (two LU solves) or, on tiny levels, as
  one Kronecker system.
* Combination technique.  Lambda_+ = {l1 + l2 = L + L0}, Lambda_- =
  {l1 + l2 = L + L0 - 1}, l in [L0, L];  Sigma_hat = sum_+ - sum_-.  For
  Hermitian data Sigma_{l2 l1} = Sigma_{l1 l2}^H, so only l1 >= l2 is solved and
  off-diagonal pairs count twice (Lambda_H; the printed set union is read as an
  intersection).
* Far-field variance of component c in direction x_i:
      V_c(x_i) = sum_{Lambda_H} sign * mult * Re (FF_{l1} Sigma FF_{l2}^H)_{(c,i),(c,i)}.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import efie
from . import mesh as meshmod


# ----------------------------------------------------------------------------- covariance
def covariance(kind: str, sigma: float, ell: float, X1, N1, X2, N2) -> np.ndarray:
    """K(x, y) between point sets X1 (Q1,3) and X2 (Q2,3); N1, N2 are the
    triangle normals at those points (used by 'normal_dot').
      gaussian : sigma^2 exp(-r^2 / (2 ell^2))
      matern32 : sigma^2 (1 + sqrt3 r/ell) exp(-sqrt3 r/ell)
      constant : sigma^2
      normal_dot: sigma^2 n(x).n(y)   (rigid translation c ~ N(0, sigma^2 I))
    r is the Euclidean distance in R^3."""
    if kind == "constant":
        return np.full((len(X1), len(X2)), sigma ** 2)
    if kind == "normal_dot":
        return sigma ** 2 * (N1 @ N2.T)
    d2 = np.sum(X1 ** 2, 1)[:, None] + np.sum(X2 ** 2, 1)[None, :] - 2.0 * X1 @ X2.T
    d2 = np.maximum(d2, 0.0)
    if kind == "gaussian":
        return sigma ** 2 * np.exp(-d2 / (2.0 * ell ** 2))
    if kind == "matern32":
        a = np.sqrt(3.0 * d2) / ell
        return sigma ** 2 * (1.0 + a) * np.exp(-a)
    raise ValueError(kind)


def covariance_dell(kind: str, sigma: float, ell: float, X1, N1, X2, N2) -> np.ndarray:
    """dK/d ell (zero for 'constant' and 'normal_dot')."""
    if kind in ("constant", "normal_dot"):
        return np.zeros((len(X1), len(X2)))
    d2 = np.sum(X1 ** 2, 1)[:, None] + np.sum(X2 ** 2, 1)[None, :] - 2.0 * X1 @ X2.T
    d2 = np.maximum(d2, 0.0)
    if kind == "gaussian":
        return sigma ** 2 * np.exp(-d2 / (2.0 * ell ** 2)) * d2 / ell ** 3
    a = np.sqrt(3.0 * d2) / ell
    return sigma ** 2 * a * a * np.exp(-a) / ell


# ----------------------------------------------------------------------------- levels
@dataclass
class Level:
    mesh: meshmod.RWGMesh
    k: float
    Z: np.ndarray
    lu: tuple
    u: np.ndarray              # first-moment coefficients (ne,)
    X: np.ndarray              # quadrature nodes (Q,3), Q = 6 nt, ordered (t, q)
    Nq: np.ndarray             # triangle normal at each node (Q,3)
    Wgt: sp.csr_matrix         # (ne, Q) shape-derivative RHS weights
    FF: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.mesh.ne


def rhs_weights(m: meshmod.RWGMesh, k: float, u: np.ndarray, field_kind: str = "radial"):
    """Wgt (ne x 6nt, sparse), nodes X (6nt,3) and normals: the map from the
    values of v_r at the quadrature nodes to the shape-derivative RHS b'."""
    X, W, Phi, D = efie.basis_at_points(m)
    ue = u[m.tri_edge]                                      # (nt,3) coefficients of local functions
    j = np.einsum("ta,taqc->tqc", ue, Phi)                  # current at the nodes (nt,6,3)
    divj = np.sum(ue * D, axis=1)                            # (nt,)
    if field_kind == "radial":
        nu = np.einsum("tqc,tc->tq", X / np.linalg.norm(X, axis=-1, keepdims=True), m.normal)
    elif field_kind == "normal":
        nu = np.ones_like(W)
    else:
        raise ValueError(field_kind)
    core = (1j / k) * divj[:, None, None] * D[:, :, None] \
        - 1j * k * np.einsum("tqc,taqc->taq", j, Phi)        # (nt,3,6)
    wloc = (W * nu)[:, None, :] * core                      # (nt,3,6)
    nt = m.nt
    rows = np.repeat(m.tri_edge.ravel(), 6)                 # edge of (t,a), repeated over q
    cols = (6 * np.arange(nt)[:, None, None] + np.arange(6)[None, None, :]).repeat(3, axis=1).ravel()
    Wgt = sp.csr_matrix((wloc.ravel(), (rows, cols)), shape=(m.ne, 6 * nt))
    Nq = np.repeat(m.normal, 6, axis=0)
    return Wgt, X.reshape(-1, 3), Nq


def make_level(V, F, k: float, d=(0.0, 0.0, 1.0), pol=(1.0, 0.0, 0.0), field_kind: str = "radial",
               n_gauss: int = 5, Z: np.ndarray | None = None) -> Level:
    m = meshmod.build(V, F)
    if Z is None:
        Z = efie.assemble(m, k, n_gauss=n_gauss)
    lu = sla.lu_factor(Z)
    b = efie.incident_rhs(m, k, np.asarray(d, float), np.asarray(pol))
    u = sla.lu_solve(lu, b)
    Wgt, X, Nq = rhs_weights(m, k, u, field_kind)
    return Level(m, k, Z, lu, u, X, Nq, Wgt, extra={"b": b})


def rhs_correlation(l1: Level, l2: Level, kind: str, sigma: float, ell: float, chunk: int = 8192) -> np.ndarray:
    """C_{l1 l2} = Wgt1 K Wgt2^H  (N1 x N2)."""
    W2H = l2.Wgt.conj().T.tocsc()
    C = np.zeros((l1.n, l2.n), dtype=np.complex128)
    Q1 = l1.X.shape[0]
    W1 = l1.Wgt.tocsc()
    for q0 in range(0, Q1, chunk):
        sl = slice(q0, min(Q1, q0 + chunk))
        K = covariance(kind, sigma, ell, l1.X[sl], l1.Nq[sl], l2.X, l2.Nq)
        C += W1[:, sl] @ (W2H.T @ K.T).T
    return C


def two_sided_solve(l1: Level, l2: Level, C: np.ndarray) -> np.ndarray:
    """Sigma with Z1 Sigma Z2^H = C: Y = Z1^{-1} C, Sigma^H = Z2^{-1} Y^H."""
    Y = sla.lu_solve(l1.lu, C)
    return sla.lu_solve(l2.lu, Y.conj().T).conj().T


def full_tensor_solve(Z1: np.ndarray, Z2: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Sigma from the Kronecker system (Z1 (x) conj Z2) vec Sigma = vec C
    (row-major vec).  Tiny levels only: N1*N2 unknowns."""
    A = np.kron(Z1, Z2.conj())
    return np.linalg.solve(A, C.ravel()).reshape(C.shape)


# ----------------------------------------------------------------------------- combination technique
def ct_pairs(L0: int, L: int) -> list[tuple[int, int, int, int]]:
    """Hermitian-reduced index set Lambda_H: (l1, l2, sign, mult) with l1 >= l2,
    sign +1 on l1+l2 = L+L0, -1 on l1+l2 = L+L0-1, mult 2 when l1 != l2.
    Ordered by sign (Lambda_+ first) then by descending l1."""
    out = []
    for sgn, tot in ((1, L + L0), (-1, L + L0 - 1)):
        for l1 in range(L, L0 - 1, -1):
            l2 = tot - l1
            if L0 <= l2 <= l1:
                out.append((l1, l2, sgn, 1 if l1 == l2 else 2))
    return out


def ct_pairs_full(L0: int, L: int) -> list[tuple[int, int, int]]:
    """Full index set Lambda (ordered pairs) with signs."""
    out = []
    for sgn, tot in ((1, L + L0), (-1, L + L0 - 1)):
        for l1 in range(L0, L + 1):
            l2 = tot - l1
            if L0 <= l2 <= L:
                out.append((l1, l2, sgn))
    return out


def ct_dofs(N: dict[int, int], L0: int, L: int) -> dict[str, float]:
    """Bookkeeping: N_hat over Lambda_H (each unordered pair once) and over
    Lambda, the largest block, and the efficiencies N_L^2 / N_hat."""
    nh = sum(N[a] * N[b] for a, b, s, m in ct_pairs(L0, L))
    nfull = sum(N[a] * N[b] for a, b, s in ct_pairs_full(L0, L))
    nmax = max(N[a] * N[b] for a, b, s in ct_pairs_full(L0, L))
    NL2 = float(N[L]) ** 2
    return {"N_hat_H": nh, "N_hat": nfull, "N_hat_max": nmax,
            "eff_H": NL2 / nh, "eff": NL2 / nfull, "eff_max": NL2 / nmax}


# ----------------------------------------------------------------------------- far field
def far_field_matrix(l: Level, xh: np.ndarray) -> np.ndarray:
    return efie.far_field_matrix(l.mesh, l.k, xh)


def pair_variance(FF1: np.ndarray, Sigma: np.ndarray, FF2: np.ndarray) -> np.ndarray:
    """Re diag(FF1 Sigma FF2^H) per component: (3, n_a)."""
    P = np.einsum("cim,mn->cin", FF1, Sigma)
    return np.real(np.einsum("cin,cin->ci", P, FF2.conj()))


def pair_correlation(FF1: np.ndarray, Sigma: np.ndarray, FF2: np.ndarray) -> np.ndarray:
    """(FF1 Sigma FF2^H) per component: (3, n_a, n_a)."""
    return np.einsum("cim,mn,cjn->cij", FF1, Sigma, FF2.conj())


def far_field_moments(levels: dict[int, Level], blocks: dict[tuple[int, int], np.ndarray],
                      L0: int, L: int, xh: np.ndarray):
    """CT far-field variance V (3, n_a) and the per-pair contributions."""
    FF = {s: far_field_matrix(levels[s], xh) for s in levels}
    V = np.zeros((3, xh.shape[0]))
    per = {}
    for l1, l2, sgn, mult in ct_pairs(L0, L):
        per[(l1, l2)] = pair_variance(FF[l1], blocks[(l1, l2)], FF[l2])
        V += sgn * mult * per[(l1, l2)]
    return V, per


def near_field_moments(levels: dict[int, Level], blocks: dict[tuple[int, int], np.ndarray],
                       L0: int, L: int, P: np.ndarray):
    """CT variance of the shape derivative of the scattered field at field
    points P (n_p, 3): Var[E'_c](P_p) = sum_pairs sign*mult*Re (NF1 Sigma NF2^H)
    at ((c,p),(c,p)) (3, n_p), and the finest level's mean field E^sc (3, n_p).
    Same combination as far_field_moments, with the near-field map."""
    NF = {s: efie.near_field_matrix(levels[s].mesh, levels[s].k, P) for s in levels}
    V = np.zeros((3, P.shape[0]))
    for l1, l2, sgn, mult in ct_pairs(L0, L):
        V += sgn * mult * pair_variance(NF[l1], blocks[(l1, l2)], NF[l2])
    mean = np.einsum("cpm,m->cp", NF[L], levels[L].u)
    return V, mean


def rcs_db(V: np.ndarray, pol_norm2: float = 1.0) -> np.ndarray:
    """Display transform of a (non-negative) far-field power: 10 log10(4 pi V/|p|^2)
    (the paper's RCS definition applied literally; negative CT values clamp)."""
    return 10.0 * np.log10(4.0 * np.pi * np.maximum(V, 1e-300) / pol_norm2)


# ----------------------------------------------------------------------------- whole pipeline
def second_moment(meshes: dict[int, tuple[np.ndarray, np.ndarray]], k: float, L0: int, L: int,
                  kind: str, sigma: float, ell: float, xh: np.ndarray, d=(0.0, 0.0, 1.0),
                  pol=(1.0, 0.0, 0.0), field_kind: str = "radial", n_gauss: int = 5,
                  levels: dict[int, Level] | None = None):
    """Full FOSB second moment over the CT index set.  Returns (V, per-pair V,
    blocks, C blocks, levels)."""
    if levels is None:
        levels = {s: make_level(*meshes[s], k, d, pol, field_kind, n_gauss) for s in range(L0, L + 1)}
    Cs, blocks = {}, {}
    for l1, l2, sgn, mult in ct_pairs(L0, L):
        Cs[(l1, l2)] = rhs_correlation(levels[l1], levels[l2], kind, sigma, ell)
        blocks[(l1, l2)] = two_sided_solve(levels[l1], levels[l2], Cs[(l1, l2)])
    V, per = far_field_moments(levels, blocks, L0, L, xh)
    return V, per, blocks, Cs, levels


# ----------------------------------------------------------------------------- gradient
def adjoint_maps(l: Level, xh: np.ndarray) -> np.ndarray:
    """P_l = FF_l Z_l^{-1} Wgt_l  (3 n_a x Q_l)."""
    FF = far_field_matrix(l, xh).reshape(-1, l.n)
    R = sla.lu_solve(l.lu, FF.T, trans=1).T                # FF Z^{-1}
    return np.asarray((l.Wgt.T @ R.T).T)


def variance_adjoint_route(levels: dict[int, Level], L0: int, L: int, kind: str, sigma: float, ell: float,
                           xh: np.ndarray) -> np.ndarray:
    """CT far-field variance (3, n_a) without Sigma blocks: V is linear in
    C = Wgt1 K Wgt2^H, so with P_l = FF_l Z_l^{-1} Wgt_l
        V_r = sum_pairs sign*mult*Re (P_l1 K P_l2^H)[r, r]."""
    P = {s: adjoint_maps(levels[s], xh) for s in levels}
    V = np.zeros(3 * xh.shape[0])
    for l1, l2, sgn, mult in ct_pairs(L0, L):
        a, b = levels[l1], levels[l2]
        K = covariance(kind, sigma, ell, a.X, a.Nq, b.X, b.Nq)
        V += sgn * mult * np.real(np.sum((P[l1] @ K) * P[l2].conj(), axis=1))
    return V.reshape(3, -1)


def summed_variance_and_gradient(levels: dict[int, Level], L0: int, L: int, kind: str, sigma: float,
                                 ell: float, xh: np.ndarray, weights: np.ndarray | None = None):
    """S = sum_{c,i} g_{c,i} V_c(x_i) (g = 1 unless weights (3, n_a) are given)
    and (dS/dsigma, dS/dell) through the linearity of S in K:
        S = sum_pairs sign*mult*Re sum_ab K_ab G_ab,  G = P1^T diag(g) conj(P2)."""
    P = {s: adjoint_maps(levels[s], xh) for s in levels}
    g = np.ones(3 * xh.shape[0]) if weights is None else np.asarray(weights, dtype=np.float64).reshape(-1)
    S = 0.0
    dsig = 0.0
    dell = 0.0
    for l1, l2, sgn, mult in ct_pairs(L0, L):
        G = P[l1].T @ (g[:, None] * P[l2].conj())
        a, b = levels[l1], levels[l2]
        K = covariance(kind, sigma, ell, a.X, a.Nq, b.X, b.Nq)
        dK = covariance_dell(kind, sigma, ell, a.X, a.Nq, b.X, b.Nq)
        S += sgn * mult * np.real(np.sum(K * G))
        dsig += sgn * mult * np.real(np.sum((2.0 / sigma) * K * G))
        dell += sgn * mult * np.real(np.sum(dK * G))
    return S, np.array([dsig, dell])
