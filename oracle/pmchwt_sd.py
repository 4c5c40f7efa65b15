"""Shape derivative of the dielectric problem: its right-hand side on the
Galerkin PMCHWT system (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper states the DE shape derivative as a PMCHWT solve with data built
from the jumps of the field across the boundary (FOA section, the DE
shape-derivative equation).  Its printed data are garbled, so they are derived
here (non-magnetic interior, mu_r = 1, the paper's material in every
experiment).  For a normal perturbation v = v_n n of the boundary the shape
derivatives E'^0 (outside, radiating, no incident part) and E'^1 (inside)
solve Maxwell's equations in each medium with the jumps
    a = n x (E'^0 - E'^1) = grad_G(v_n [E_n]) x n,
    b = n x (H~'^0 - H~'^1) = i k0 (1 - eps_r) v_n E_t,
obtained by differentiating the transmission conditions along the flow:
n x [E'] = grad_G v_n x n [E_n] - v_n n x [d_n E], with
n x d_n E = n x grad_G E_n + (curl E)_t, [(curl E)_t] = i k0 (1 - mu_r) H~_t = 0,
[(curl H~)_t] = -i k0 (1 - eps_r) E_t, [H~_n] = 0 and [E_n] = (1 - 1/eps_r) E^0_n.
On the exterior traces (J = n x H~, M = -n x E of oracle/pmchwt.py):
    E^0_n = -(i/k0) div_G J,    E_t = n x M.

With J1 = J0 - b and M1 = M0 + a the interior extinction statement moves the
jumps to the right-hand side: the derivative's exterior traces solve the same
PMCHWT system Z [J'; M'] = [r_E; r_H] with
    r_E = -eta <E_k1 b> - <H_k1 a> + 1/2 <n x a>,
    r_H = -<H_k1 b> + <E_k1 a> / eta + 1/2 <n x b>,
<X>[m] = int phi_m . X (principal values; the halves are the identity parts of
the interior potentials' exterior traces, which no longer cancel).  Written
with psi = v_n [E_n] (a = curl_G psi is solenoidal) and moved onto the kernel
by parts:
    <n x a>   = -int psi div phi_m,
    <E_k a>   = i k int int phi_m(x) . (grad_x G x n_y) psi(y),
    <H_k a>   = k^2 int int G phi_m(x) . n_y psi(y) - int int div phi_m(x) (grad_x G . n_y) psi(y),
    <E_k b>   = i k int int G phi_m . b(y) - (i/k) int int div phi_m(x) grad_x G . b(y),
    <H_k b>   = int int phi_m(x) . (grad_x G x b(y)),
all at the interior wavenumber k1.

The perturbation amplitude enters through its values at the 6-point nodes of
every triangle (as on the PEC path): the right-hand side is W v with W
(2N x 6 nt).  Non-touching triangle pairs integrate x with the 6-point rule and
take the source at the nodes; touching pairs use the Sauter-Schwab points and
the amplitude's quadratic interpolant through the triangle's six nodes.
"""

from __future__ import annotations

import numpy as np

from . import efie
from . import mesh as meshmod
from . import pmchwt
from .quadrature import chi, sauter_schwab, touching_order, triangle_rule6
from .uq import ct_pairs


def green(k, R):
    return np.exp(1j * k * R) / (4.0 * np.pi * R)


def lagrange6():
    """Coefficients of the quadratic Lagrange basis through the 6-point rule's
    nodes, in the monomials (1, l1, l2, l1^2, l1 l2, l2^2) of the barycentric
    coordinates l1, l2: ell_q(l) = mono(l) @ Cinv[:, q]."""
    bary, _ = triangle_rule6()
    l1, l2 = bary[:, 1], bary[:, 2]
    V = np.stack([np.ones(6), l1, l2, l1 * l1, l1 * l2, l2 * l2], axis=1)
    return np.linalg.inv(V)


def _mono(l1, l2):
    return np.stack([np.ones_like(l1), l1, l2, l1 * l1, l1 * l2, l2 * l2], axis=-1)


def node_data(m: meshmod.RWGMesh, k0: float, eps_r: float, u: np.ndarray):
    """Per triangle: c_psi = (1 - 1/eps_r) E^0_n (constant on the triangle),
    and the coefficients of E_t = n x M as a function on it: E_t(y) = sum_a
    uM_a n x phi_a(y).  Returns (c_psi (nt,), uM_loc (nt, 3))."""
    ne = m.ne
    uJ, uM = u[:ne], u[ne:]
    div = meshmod.rwg_div(m, np.arange(m.nt)[:, None], np.arange(3)[None, :])          # (nt,3)
    divJ = np.sum(div * uJ[m.tri_edge], axis=1)
    En = -1j / k0 * divJ
    return (1.0 - 1.0 / eps_r) * En, uM[m.tri_edge]


def _et(m, j, uMl, y):
    """E_t(y) = n_j x M(y) on triangle j (y (..., 3)), M = sum_a uM_a phi_a."""
    a = np.arange(3)
    ph = meshmod.rwg_eval(m, np.full(3, j), a, y[..., None, :])                        # (...,3,3)
    Mv = np.einsum("...ac,a->...c", ph, uMl[j])
    return np.cross(m.normal[j], Mv)


def rhs_matrix(m: meshmod.RWGMesh, k0: float, eps_r: float, u: np.ndarray, n_gauss: int = 5) -> np.ndarray:
    """W (2N x 6 nt): the shape-derivative right-hand side [r_E; r_H] = W v for
    the amplitude values v at the 6-point nodes (node 6 j + q of triangle j),
    for the first moment u = [J; M] of one incidence.  mu_r = 1."""
    k1, eta = pmchwt.wavenumbers(k0, eps_r, 1.0)
    cb = 1j * k0 * (1.0 - eps_r)
    nt, ne = m.nt, m.ne
    X, Wq, Phi, D = efie.basis_at_points(m)               # nodes (nt,6,3), weights (nt,6), RWG values, divergences
    cpsi, uMl = node_data(m, k0, eps_r, u)
    Cinv = lagrange6()
    tp = meshmod.touching_pairs(m)
    touch = {}
    for kind, pairs in tp.items():
        for i, j in pairs:
            touch[(int(i), int(j))] = kind
    # local blocks per (test triangle i, source triangle j): rE[a][q], rH[a][q]
    WE = np.zeros((nt, 3, nt, 6), dtype=complex)
    WH = np.zeros((nt, 3, nt, 6), dtype=complex)
    xs, ys, ws = {}, {}, {}
    for kind in ("identical", "edge", "vertex"):
        xs[kind], ys[kind], ws[kind] = sauter_schwab(kind, n_gauss)
    ET = np.stack([_et(m, j, uMl, X[j]) for j in range(nt)])                     # (nt,6q,3): E_t at the nodes
    for i in range(nt):
        # non-touching source triangles: 6-point rule in x, sources at the nodes
        J = np.array([j for j in range(nt) if (i, j) not in touch], dtype=np.int64)
        d = X[i][None, :, None, :] - X[J][:, None, :, :]                            # (nJ,6p,6q,3)
        R = np.linalg.norm(d, axis=-1)
        w = Wq[i][None, :, None] * Wq[J][:, None, :]                                # (nJ,6,6)
        G = green(k1, R) * w
        gG = ((1j * k1 * R - 1.0) * np.exp(1j * k1 * R) / (4 * np.pi * R ** 3) * w)[..., None] * d
        nJ = m.normal[J]                                                           # (nJ,3)
        etq = ET[J]                                                                # (nJ,6q,3)
        cp = cpsi[J][:, None]                                                      # (nJ,1)
        # a-terms (psi = v c_psi on the source triangle)
        EA = 1j * k1 * np.einsum("apc,jpqc->jaq", Phi[i], np.cross(gG, nJ[:, None, None, :]), optimize=True) * cp[:, None, :]
        HA = (k1 ** 2 * np.einsum("apc,jc,jpq->jaq", Phi[i], nJ, G, optimize=True)
              - D[i][None, :, None] * np.einsum("jpqc,jc->jq", gG, nJ, optimize=True)[:, None, :]) * cp[:, None, :]
        # b-terms (b = cb v E_t at the source node)
        EB = cb * (1j * k1 * np.einsum("apc,jqc,jpq->jaq", Phi[i], etq, G, optimize=True)
                   - (1j / k1) * D[i][None, :, None] * np.einsum("jpqc,jqc->jq", gG, etq, optimize=True)[:, None, :])
        HB = cb * np.einsum("apc,jpqc->jaq", Phi[i], np.cross(gG, etq[:, None, :, :]), optimize=True)
        WE[i][:, J, :] += np.transpose(-eta * EB - HA, (1, 0, 2))
        WH[i][:, J, :] += np.transpose(-HB + EA / eta, (1, 0, 2))
        # touching source triangles: Sauter-Schwab points, quadratic interpolant of the amplitude
        for j in [j for j in range(nt) if (i, j) in touch]:
            kind = touch[(i, j)]
            nj = m.normal[j]
            oi, oj = touching_order(m.F[i], m.F[j])
            Pi, Pj = m.V[oi], m.V[oj]
            x = chi(Pi[0], Pi[1], Pi[2], xs[kind])                                  # (M,3)
            y = chi(Pj[0], Pj[1], Pj[2], ys[kind])
            w = ws[kind] * (2.0 * m.area[i]) * (2.0 * m.area[j])
            f = meshmod.rwg_eval(m, np.full((3, 1), i), np.arange(3)[:, None], x[None, :, :])   # (3,M,3)
            et = _et(m, j, uMl, y)                                                  # (M,3)
            T = m.V[m.F[j]]
            A = np.stack([T[1] - T[0], T[2] - T[0]], axis=1)
            lam = np.linalg.lstsq(A, (y - T[0]).T, rcond=None)[0].T                 # (M,2)
            ell = _mono(lam[:, 0], lam[:, 1]) @ Cinv                                # (M,6q)
            dd = x - y
            R = np.linalg.norm(dd, axis=-1)
            G = green(k1, R) * w
            gG = ((1j * k1 * R - 1.0) * np.exp(1j * k1 * R) / (4 * np.pi * R ** 3) * w)[:, None] * dd
            fdot = lambda v: np.sum(f * v[None], axis=-1)                           # (3,M): phi_a(x) . v
            EA = 1j * k1 * (fdot(np.cross(gG, nj)) @ ell) * cpsi[j]
            HA = (k1 ** 2 * ((fdot(np.broadcast_to(nj, dd.shape)) * G) @ ell)
                  - D[i][:, None] * ((gG @ nj) @ ell)[None, :]) * cpsi[j]
            EB = cb * (1j * k1 * ((fdot(et) * G) @ ell)
                       - (1j / k1) * D[i][:, None] * (np.sum(gG * et, axis=-1) @ ell)[None, :])
            HB = cb * (fdot(np.cross(gG, et)) @ ell)
            WE[i, :, j, :] += -eta * EB - HA
            WH[i, :, j, :] += -HB + EA / eta
        # identity terms (test and source on triangle i, 6-point rule)
        WE[i, :, i, :] += 0.5 * (-(cpsi[i] * D[i][:, None] * Wq[i][None, :]))
        WH[i, :, i, :] += 0.5 * cb * np.einsum("aqc,qc,q->aq", Phi[i], np.cross(m.normal[i], ET[i]), Wq[i])
    S = efie.incidence(m)
    WEm = S @ WE.reshape(3 * nt, 6 * nt)
    WHm = S @ WH.reshape(3 * nt, 6 * nt)
    return np.vstack([np.asarray(WEm), np.asarray(WHm)])


def first_order_far_field(m: meshmod.RWGMesh, k0: float, eps_r: float, Z: np.ndarray, u: np.ndarray,
                          vnodes: np.ndarray, xh: np.ndarray, n_gauss: int = 5) -> np.ndarray:
    """F' (n_a, 3) of the shape derivative for amplitude values vnodes (6 nt)."""
    W = rhs_matrix(m, k0, eps_r, u, n_gauss)
    du = np.linalg.solve(Z, W @ vnodes)
    return pmchwt.far_field(m, k0, du, xh)


# ----------------------------------------------------------------------------- second moment
class Level:
    """A dielectric level for the shape-uncertainty second moment: PMCHWT
    matrix and LU, first moment u = [J; M], quadrature nodes X and normals Nq,
    the right-hand-side map Wgt = W diag(nu) (2N x 6 nt) from the amplitude at
    the nodes (nu = (x/|x|).n for the radial field, 1 for the normal field)."""

    def __init__(self, V, F, k0: float, eps_r: float, d, pol, field_kind: str = "radial", n_gauss: int = 5):
        import scipy.linalg as sla
        self.mesh = m = meshmod.build(V, F)
        self.k0, self.eps_r = k0, eps_r
        self.Z = pmchwt.assemble(m, k0, eps_r, 1.0, n_gauss)
        self.lu = sla.lu_factor(self.Z)
        self.b = pmchwt.incident_rhs(m, k0, d, pol)
        self.u = sla.lu_solve(self.lu, self.b)
        X, Wq, _, _ = efie.basis_at_points(m)
        if field_kind == "radial":
            nu = np.einsum("tqc,tc->tq", X / np.linalg.norm(X, axis=-1, keepdims=True), m.normal)
        elif field_kind == "normal":
            nu = np.ones_like(Wq)
        else:
            raise ValueError(field_kind)
        self.Wgt = rhs_matrix(m, k0, eps_r, self.u, n_gauss) * nu.ravel()[None, :]
        self.X = X.reshape(-1, 3)
        self.Nq = np.repeat(m.normal, 6, axis=0)

    @property
    def n(self) -> int:
        return 2 * self.mesh.ne


def second_moment(levels: dict, L0: int, L: int, kind: str, sigma: float, ell: float, xh: np.ndarray):
    """CT far-field variance (3, n_a) of the dielectric shape derivative:
    C = Wgt1 K Wgt2^H with K the amplitude covariance at the nodes of both
    levels, the two-sided solve and the PMCHWT far-field contraction.
    Returns (V, blocks)."""
    import scipy.linalg as sla
    from .uq import covariance
    FF = {s: pmchwt.far_field_matrix(levels[s].mesh, levels[s].k0, xh) for s in levels}
    V = np.zeros((3, xh.shape[0]))
    blocks = {}
    for l1, l2, sgn, mult in ct_pairs(L0, L):
        a, b = levels[l1], levels[l2]
        K = covariance(kind, sigma, ell, a.X, a.Nq, b.X, b.Nq)
        C = a.Wgt @ K @ b.Wgt.conj().T
        Y = sla.lu_solve(a.lu, C)
        Sig = sla.lu_solve(b.lu, Y.conj().T).conj().T
        blocks[(l1, l2)] = Sig
        V += sgn * mult * np.real(np.einsum("cim,mn,cin->ci", FF[l1], Sig, FF[l2].conj()))
    return V, blocks
