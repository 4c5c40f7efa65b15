"""Pins of the low-rank covariance (oracle/lowrank.py): properties of the
pivoted Cholesky factor, the Nystrom extension against the factor's own
columns, exact ranks of the separable models, and convergence of the
low-rank second moment to the dense one (CPU)."""

import numpy as np
import pytest

import workloads
from oracle import lowrank, uq

SIG, ELL = 0.01, 0.5


def test_pivoted_cholesky_properties(oracle_levels):
    lv = oracle_levels(1)
    X, N = lv.X, lv.Nq
    K = uq.covariance("gaussian", SIG, ELL, X, N, X, N)
    piv, L, res = lowrank.pivoted_cholesky("gaussian", SIG, ELL, X, N, len(X), 1e-10)
    R = K - L @ L.T
    s2 = SIG ** 2
    assert len(set(piv.tolist())) == len(piv) and res <= 1e-10
    assert np.abs(R[piv]).max() < 1e-13 * s2                      # exact on the pivot rows
    dres = np.diag(R)
    assert dres.min() > -1e-14 * s2 and dres.max() <= 1e-10 * s2 * (1 + 1e-6)
    assert np.abs(R).max() <= dres.max() * (1 + 1e-6) + 1e-16     # PSD residual: |R_ij| <= sqrt(R_ii R_jj)
    # each pivot was the largest remaining diagonal entry when it was taken
    d = np.full(len(X), s2)
    for j, p in enumerate(piv):
        assert d[p] >= (1 - 1e-9) * d.max() - 1e-30
        d = d - L[:, j] ** 2
        d[p] = 0.0


def test_nystrom_equals_the_factor(oracle_levels):
    """K(X, P) K(P, P)^{-1} K(P, X) (direct formula) equals L L^T of the
    pivoted Cholesky factor, and K(X, P) L[P]^{-T} equals L."""
    lv = oracle_levels(1)
    X, N = lv.X, lv.Nq
    piv, L, _ = lowrank.pivoted_cholesky("matern32", SIG, ELL, X, N, 120, 1e-6)
    Kr = lowrank.nystrom("matern32", SIG, ELL, X, N, X, N, X[piv], N[piv])
    assert np.abs(Kr - L @ L.T).max() < 1e-9 * SIG ** 2
    Phi = np.linalg.solve(L[piv], uq.covariance("matern32", SIG, ELL, X[piv], N[piv], X, N)).T
    assert np.abs(Phi - L).max() < 1e-8 * SIG


@pytest.mark.parametrize("kind,rank", [("constant", 1), ("normal_dot", 3)])
def test_separable_models_have_exact_rank(oracle_levels, kind, rank):
    """sigma^2 (rank 1) and sigma^2 n(x).n(y) (rank 3): the factor on the
    ladder's nodes stops at that rank and the low-rank CT variance equals the
    dense one."""
    xh = workloads.angles_xz(19)
    levels = {s: oracle_levels(s) for s in (0, 1, 2)}
    X, N, off = lowrank.ladder_candidates(levels, 0, 2)
    piv, L, res = lowrank.pivoted_cholesky(kind, SIG, ELL, X, N, 50, 1e-12)
    assert len(piv) == rank and res <= 1e-12
    V, _, _, _, _ = uq.second_moment(None, 1.0, 0, 2, kind, SIG, ELL, xh, levels=levels)
    Vr, _ = lowrank.second_moment(levels, 0, 2, xh, L, off)
    assert np.abs(Vr - V).max() < 1e-10 * np.abs(V).max()


def test_lowrank_variance_converges_to_dense(oracle_levels):
    """Gaussian covariance, CT over s = 0..2, factor on the nodes of all three
    levels: the low-rank variance approaches the dense one as tol falls, to
    about the tolerance."""
    xh = workloads.angles_xz(19)
    levels = {s: oracle_levels(s) for s in (0, 1, 2)}
    X, N, off = lowrank.ladder_candidates(levels, 0, 2)
    V, _, _, _, _ = uq.second_moment(None, 1.0, 0, 2, "gaussian", SIG, ELL, xh, levels=levels)
    errs, ranks = [], []
    for tol in (1e-3, 1e-6, 1e-9, 1e-12):
        piv, L, _ = lowrank.pivoted_cholesky("gaussian", SIG, ELL, X, N, len(X), tol)
        Vr, _ = lowrank.second_moment(levels, 0, 2, xh, L, off)
        errs.append(float(np.linalg.norm(Vr - V) / np.linalg.norm(V)))
        ranks.append(len(piv))
    assert ranks == sorted(ranks) and errs[-1] < 1e-9 and errs[0] > errs[-1] * 1e5, (ranks, errs)
