"""Low-rank covariance: pivoted Cholesky and the Nystrom extension (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names low-rank representations of the covariance as the way to
make the second-moment right-hand side cheap (future-work remarks; the
Fichera experiment's covariance is a finite sum of separable terms).  With
K(x, y) ~ sum_j phi_j(x) phi_j(y) the right-hand-side correlation factors,
C_l1l2 = (Wgt_l1 Phi_l1)(Wgt_l2 Phi_l2)^H, and so does Sigma.

The factor is built here by the greedy pivoted Cholesky decomposition of the
covariance on a candidate point set, the quadrature nodes of every level of
the ladder (so that the factor's rows are the feature vectors of all the
nodes the right-hand sides use):
    d = diag K;  at each step take the pivot p with the largest remaining d
    (the lowest index among those within a relative 1e-9 of the largest, so
    that near-ties are decided the same way in any rounding order), form the
    column  L[:, j] = (K(X, x_p) - L[:, :j] L[p, :j]^T) / sqrt(d_p),  update
    d -= L[:, j]^2 and set d_p = 0;  stop when the largest d is at most
    tol * max(diag K) or the rank reaches max_rank.
On the pivots P the factor reproduces K exactly (L[P] L[P]^T = K(P, P));
on the other candidates it is the Nystrom approximation
    K_r(x, y) = K(x, P) K(P, P)^{-1} K(P, y),
whose error on the candidates is bounded by the largest remaining diagonal
entry.  The low-rank second moment uses K_r = L_l1 L_l2^T, with L_l the rows
of the factor that belong to level l.
"""

from __future__ import annotations

import numpy as np

from . import uq

TIE = 1e-9


def _cov(kind, sigma, ell, X1, N1, X2, N2):
    return uq.covariance(kind, sigma, ell, X1, N1, X2, N2)


def pivoted_cholesky(kind: str, sigma: float, ell: float, X: np.ndarray, N: np.ndarray, max_rank: int,
                     tol: float):
    """Greedy pivoted Cholesky of K(X, X).  Returns (pivots (r,), L (n, r),
    residual = largest remaining diagonal / largest initial diagonal)."""
    n = X.shape[0]
    d = np.array([_cov(kind, sigma, ell, X[i:i + 1], N[i:i + 1], X[i:i + 1], N[i:i + 1])[0, 0]
                  for i in range(n)]) if kind == "normal_dot" else np.full(n, float(sigma) ** 2)
    dmax0 = d.max()
    L = np.zeros((n, max_rank))
    piv = []
    for j in range(max_rank):
        dmax = d.max()
        if dmax <= tol * dmax0:
            break
        p = int(np.nonzero(d >= (1.0 - TIE) * dmax)[0][0])
        col = _cov(kind, sigma, ell, X, N, X[p:p + 1], N[p:p + 1])[:, 0] - L[:, :j] @ L[p, :j]
        L[:, j] = col / np.sqrt(d[p])
        d = d - L[:, j] ** 2
        d[p] = 0.0
        piv.append(p)
    r = len(piv)
    return np.array(piv, dtype=np.int64), L[:, :r], (d.max() / dmax0 if r else 1.0)


def ladder_candidates(levels: dict[int, uq.Level], L0: int, L: int):
    """Candidate points: the quadrature nodes of levels L0..L in that order,
    their triangle normals, and the offset of each level's rows."""
    X = np.concatenate([levels[s].X for s in range(L0, L + 1)])
    N = np.concatenate([levels[s].Nq for s in range(L0, L + 1)])
    off, o = {}, 0
    for s in range(L0, L + 1):
        off[s] = o
        o += levels[s].X.shape[0]
    return X, N, off


def nystrom(kind: str, sigma: float, ell: float, X1, N1, X2, N2, P, NP) -> np.ndarray:
    """K_r(X1, X2) = K(X1, P) K(P, P)^{-1} K(P, X2)."""
    Kpp = _cov(kind, sigma, ell, P, NP, P, NP)
    return _cov(kind, sigma, ell, X1, N1, P, NP) @ np.linalg.solve(Kpp, _cov(kind, sigma, ell, P, NP, X2, N2))


def second_moment(levels: dict[int, uq.Level], L0: int, L: int, xh: np.ndarray, Lf: np.ndarray,
                  off: dict[int, int]):
    """CT variance (3, n_a) and Sigma blocks with the low-rank covariance
    K_r = L_l1 L_l2^T (Lf: the factor on the ladder's candidates, off: each
    level's first row): C_r = Wgt1 K_r Wgt2^H, the two-sided solve and the
    far-field contraction, as in the dense route."""
    blocks = {}
    for l1, l2, sgn, mult in uq.ct_pairs(L0, L):
        a, b = levels[l1], levels[l2]
        F1 = Lf[off[l1]:off[l1] + a.X.shape[0]]
        F2 = Lf[off[l2]:off[l2] + b.X.shape[0]]
        C = np.asarray(a.Wgt @ F1) @ np.asarray(b.Wgt @ F2).conj().T
        blocks[(l1, l2)] = uq.two_sided_solve(a, b, C)
    V, _ = uq.far_field_moments(levels, blocks, L0, L, xh)
    return V, blocks
