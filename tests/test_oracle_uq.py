"""Pins of the oracle's second-moment pipeline (CPU)."""

import numpy as np
import pytest

import workloads
from oracle import efie, mie, uq


def _rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def test_two_sided_solve_equals_kronecker_system(oracle_levels):
    """(Z1 (x) conj Z2) vec Sigma = vec C solved as one dense system (tiny
    levels) equals the two-sided solve."""
    l1, l0 = oracle_levels(1), oracle_levels(0)
    for a, b in ((l1, l0), (l0, l1), (l0, l0)):
        C = uq.rhs_correlation(a, b, "gaussian", 0.01, 0.5)
        S = uq.two_sided_solve(a, b, C)
        K = uq.full_tensor_solve(a.Z, b.Z, C)
        assert _rel(S, K) < 1e-12


def test_rank_one_rhs_gives_rank_one_sigma(oracle_levels):
    """The sphere experiment's closed form: M2[f] = f (x) f gives M2[xi] = xi (x) xi;
    here C = b b^H  =>  Sigma = u u^H with Z u = b."""
    lv = oracle_levels(2)
    b = lv.extra["b"]
    S = uq.two_sided_solve(lv, lv, np.outer(b, b.conj()))
    assert _rel(S, np.outer(lv.u, lv.u.conj())) < 1e-12


def test_rhs_correlation_hermitian_and_psd(oracle_levels):
    l2, l1 = oracle_levels(2), oracle_levels(1)
    C = uq.rhs_correlation(l2, l2, "gaussian", 0.01, 0.5)
    assert np.abs(C - C.conj().T).max() < 1e-14 * np.abs(C).max()
    ev = np.linalg.eigvalsh(0.5 * (C + C.conj().T))
    assert ev.min() > -1e-12 * ev.max()
    C21 = uq.rhs_correlation(l2, l1, "matern32", 0.01, 0.5)
    C12 = uq.rhs_correlation(l1, l2, "matern32", 0.01, 0.5)
    assert np.abs(C21 - C12.conj().T).max() < 1e-14 * np.abs(C21).max()


def test_sigma_hermitian_pairs(oracle_levels):
    """Sigma_{l2 l1} = Sigma_{l1 l2}^H up to the (tiny) asymmetry of Z."""
    l2, l1 = oracle_levels(2), oracle_levels(1)
    C21 = uq.rhs_correlation(l2, l1, "gaussian", 0.01, 0.5)
    S21 = uq.two_sided_solve(l2, l1, C21)
    S12 = uq.two_sided_solve(l1, l2, C21.conj().T)
    assert _rel(S12, S21.conj().T) < 1e-12
    C22 = uq.rhs_correlation(l2, l2, "gaussian", 0.01, 0.5)
    S22 = uq.two_sided_solve(l2, l2, C22)
    assert _rel(S22, S22.conj().T) < 1e-12
    ev = np.linalg.eigvalsh(0.5 * (S22 + S22.conj().T))
    assert ev.min() > -1e-10 * ev.max()


def test_translation_identity(oracle_levels):
    """Rigid translation c ~ N(0, sigma^2 I): K = sigma^2 n(x).n(y) and
    F_c = exp(i k (d - x).c) F, so Var[F'_c](x) -> sigma^2 k^2 |d - x|^2 |F_c(x)|^2
    as h -> 0.  Pins the sign and scale of both shape-derivative terms."""
    xh = workloads.angles_xz(37)
    d = np.array([0.0, 0.0, 1.0])
    errs = []
    for s in (1, 2, 3):
        lv = oracle_levels(s, 1.0, "normal")
        C = uq.rhs_correlation(lv, lv, "normal_dot", 1.0, 1.0)
        FF = uq.far_field_matrix(lv, xh)
        V = uq.pair_variance(FF, uq.two_sided_solve(lv, lv, C), FF)
        F = efie.far_field(lv.mesh, 1.0, lv.u, xh)
        ref = (np.sum((d[None] - xh) ** 2, 1))[:, None] * np.abs(F) ** 2
        errs.append(_rel(V.T, ref))
    assert errs[-1] < 2e-2 and errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_breathing_mode_vs_mie(oracle_levels):
    """Constant covariance sigma^2 on a radial field = random radius change:
    Var[F'_c] -> sigma^2 |dF_c/da|^2 of the exact Mie series."""
    xh = workloads.angles_xz(37)
    dF = mie.pec_far_field_radius_derivative(1.0, 1.0, xh)
    errs = []
    for s in (1, 2, 3):
        lv = oracle_levels(s)
        C = uq.rhs_correlation(lv, lv, "constant", 1.0, 1.0)
        FF = uq.far_field_matrix(lv, xh)
        V = uq.pair_variance(FF, uq.two_sided_solve(lv, lv, C), FF)
        errs.append(_rel(V.T, np.abs(dF) ** 2))
    assert errs[-1] < 3e-2 and errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_ct_index_sets():
    """Lambda_H for the workloads' ladders, and the Fichera experiment's three
    CT blocks (2,0), (1,1), (1,0) for L0=0, L=2 (Table III)."""
    assert uq.ct_pairs(1, 3) == [(3, 1, 1, 2), (2, 2, 1, 1), (2, 1, -1, 2)]
    assert uq.ct_pairs(2, 5) == [(5, 2, 1, 2), (4, 3, 1, 2), (4, 2, -1, 2), (3, 3, -1, 1)]
    assert uq.ct_pairs(0, 2) == [(2, 0, 1, 2), (1, 1, 1, 1), (1, 0, -1, 2)]
    assert uq.ct_pairs(3, 3) == [(3, 3, 1, 1)]
    assert len(uq.ct_pairs_full(2, 5)) == 7
    # Table III block dofs from N_l = 270, 792, 3204
    N = {0: 270, 1: 792, 2: 3204}
    blocks = [N[a] * N[b] for a, b, s, m in uq.ct_pairs(0, 2)]
    assert [round(x, -3) for x in blocks] == [865000, 627000, 214000]
    assert abs(blocks[0] / 8.65e5 - 1) < 1e-3 and abs(blocks[1] / 6.27e5 - 1) < 1e-3
    # kite experiment: N_L^2 / N_hat = 6.02 and N_L^2 / N_hat^max = 12.76 from the printed totals
    assert round(3.24e8 / 5.38e7, 2) == 6.02 and round(3.24e8 / 2.54e7, 2) == 12.76
    d = uq.ct_dofs(N, 0, 2)
    assert d["N_hat_H"] == sum(blocks) and abs(d["eff_H"] - 3204 ** 2 / sum(blocks)) < 1e-12


def test_ct_hermitian_reduction_and_single_level(oracle_levels):
    """Lambda (all ordered pairs) and Lambda_H give the same variance; L = L0
    reduces to the full tensor solution on that level."""
    xh = workloads.angles_xz(19)
    levels = {s: oracle_levels(s) for s in (0, 1, 2)}
    V, per, blocks, Cs, _ = uq.second_moment(None, 1.0, 0, 2, "gaussian", 0.01, 0.5, xh, levels=levels)
    FF = {s: uq.far_field_matrix(levels[s], xh) for s in levels}
    Vf = np.zeros_like(V)
    for l1, l2, sgn in uq.ct_pairs_full(0, 2):
        C = uq.rhs_correlation(levels[l1], levels[l2], "gaussian", 0.01, 0.5)
        S = uq.two_sided_solve(levels[l1], levels[l2], C)
        P = np.einsum("cim,mn,cin->ci", FF[l1], S, FF[l2].conj())
        Vf += sgn * P.real
        assert np.abs(P.imag).max() < 1e-6 * np.abs(P).max() or l1 != l2
    assert _rel(V, Vf) < 1e-10
    V1, _, _, _, _ = uq.second_moment(None, 1.0, 2, 2, "gaussian", 0.01, 0.5, xh, levels={2: levels[2]})
    C22 = uq.rhs_correlation(levels[2], levels[2], "gaussian", 0.01, 0.5)
    S22 = uq.full_tensor_solve(levels[2].Z, levels[2].Z, C22) if levels[2].n <= 120 else \
        uq.two_sided_solve(levels[2], levels[2], C22)
    assert _rel(V1, uq.pair_variance(FF[2], S22, FF[2])) < 1e-12


def test_ct_approximates_full_tensor(oracle_levels):
    """CT with L0 = 1, L = 3 is close to the full-tensor variance on level 3
    (the paper reports CT tracking the full tensor; kite: 8.68e-4)."""
    xh = workloads.angles_xz(37)
    levels = {s: oracle_levels(s) for s in (1, 2, 3)}
    V, _, _, _, _ = uq.second_moment(None, 1.0, 1, 3, "gaussian", 0.01, 0.5, xh, levels=levels)
    FF3 = uq.far_field_matrix(levels[3], xh)
    C = uq.rhs_correlation(levels[3], levels[3], "gaussian", 0.01, 0.5)
    Vfull = uq.pair_variance(FF3, uq.two_sided_solve(levels[3], levels[3], C), FF3)
    assert _rel(V, Vfull) < 5e-2


def test_adjoint_route_and_gradient(oracle_levels):
    """S = sum V through the adjoint maps equals the Sigma route; dS/dsigma =
    2S/sigma exactly; dS/dell matches a central finite difference (h = 1e-5)."""
    xh = workloads.angles_xz(19)
    levels = {s: oracle_levels(s) for s in (0, 1, 2)}
    for kind in ("gaussian", "matern32"):
        sig, ell = 0.01, 0.5
        V, _, _, _, _ = uq.second_moment(None, 1.0, 0, 2, kind, sig, ell, xh, levels=levels)
        S, g = uq.summed_variance_and_gradient(levels, 0, 2, kind, sig, ell, xh)
        assert abs(S - V.sum()) < 1e-10 * abs(V).sum()
        assert abs(g[0] - 2 * S / sig) < 1e-12 * abs(g[0])
        h = 1e-5
        Sp, _ = uq.summed_variance_and_gradient(levels, 0, 2, kind, sig, ell + h, xh)
        Sm, _ = uq.summed_variance_and_gradient(levels, 0, 2, kind, sig, ell - h, xh)
        fd = (Sp - Sm) / (2 * h)
        assert abs(fd - g[1]) < 1e-6 * abs(g[1]), (fd, g[1])


def test_weighted_adjoint_route(oracle_levels):
    """With upstream weights g: sum g V (Sigma route) equals the adjoint-route S,
    and dS/dell matches a central difference of the Sigma route."""
    xh = workloads.angles_xz(13)
    levels = {s: oracle_levels(s) for s in (0, 1, 2)}
    g = np.random.default_rng(3).standard_normal((3, 13))
    sig, ell = 0.02, 0.4
    V, _, _, _, _ = uq.second_moment(None, 1.0, 0, 2, "gaussian", sig, ell, xh, levels=levels)
    S, grad = uq.summed_variance_and_gradient(levels, 0, 2, "gaussian", sig, ell, xh, weights=g)
    assert abs(S - np.sum(g * V)) < 1e-10 * np.sum(np.abs(g * V))
    h = 1e-5
    Vp = uq.second_moment(None, 1.0, 0, 2, "gaussian", sig, ell + h, xh, levels=levels)[0]
    Vm = uq.second_moment(None, 1.0, 0, 2, "gaussian", sig, ell - h, xh, levels=levels)[0]
    fd = np.sum(g * (Vp - Vm)) / (2 * h)
    assert abs(fd - grad[1]) < 1e-6 * abs(grad[1]), (fd, grad[1])


@pytest.mark.parametrize("kind", ["gaussian", "matern32"])
def test_full_tensor_variance_is_nonnegative(oracle_levels, kind):
    """Single-level (full tensor) variance Re diag(FF Sigma FF^H) is a variance:
    C = W K W^H is Hermitian PSD for a PSD covariance, so Sigma = Z^-1 C Z^-H is
    too, and every component at every angle is >= 0 (to rounding).  A missing
    conjugation or a sign error in W breaks positivity."""
    xh = workloads.angles_xz(61)
    for s in (1, 2):
        lv = oracle_levels(s)
        C = uq.rhs_correlation(lv, lv, kind, 0.01, 0.5)
        S = uq.two_sided_solve(lv, lv, C)
        FF = uq.far_field_matrix(lv, xh)
        V = uq.pair_variance(FF, S, FF)
        assert V.min() >= -1e-12 * V.max(), (s, V.min(), V.max())
        # the off-diagonal far-field correlation is Hermitian in the angle pair
        Cor = uq.pair_correlation(FF, S, FF)
        assert np.abs(Cor - np.conj(np.transpose(Cor, (0, 2, 1)))).max() < 1e-10 * np.abs(Cor).max()


def test_covariance_hand_values():
    """Hand-computed values of the covariance models at chosen distances
    (amplitude sigma is the standard deviation, r the Euclidean distance):
    Gaussian sigma^2 exp(-r^2/(2 ell^2)) at r = ell is sigma^2 e^{-1/2} and at
    r = 2 ell sigma^2 e^{-2}; Matern-3/2 sigma^2 (1 + sqrt3 r/ell) e^{-sqrt3 r/ell}
    at r = ell/sqrt3 is 2 sigma^2 e^{-1} and at r = 0 sigma^2; the rigid
    translation model is sigma^2 n(x).n(y)."""
    sig, ell = 0.3, 0.7
    X1 = np.array([[0.0, 0.0, 0.0]])
    dirn = np.array([0.6, 0.0, 0.8])
    pts = np.array([[0.0, 0.0, 0.0], ell * dirn, 2 * ell * dirn, ell / np.sqrt(3.0) * dirn])
    g = uq.covariance("gaussian", sig, ell, X1, None, pts, None)[0]
    assert np.allclose(g, sig ** 2 * np.array([1.0, np.exp(-0.5), np.exp(-2.0), np.exp(-1.0 / 6.0)]),
                       rtol=1e-14, atol=0)
    m = uq.covariance("matern32", sig, ell, X1, None, pts, None)[0]
    a = np.sqrt(3.0) * np.array([0.0, 1.0, 2.0, 1.0 / np.sqrt(3.0)])
    assert abs(m[3] - 2.0 * sig ** 2 * np.exp(-1.0)) < 1e-14 * sig ** 2
    assert abs(m[0] - sig ** 2) < 1e-15
    assert abs(m[1] - sig ** 2 * (1 + np.sqrt(3.0)) * np.exp(-np.sqrt(3.0))) < 1e-14 * sig ** 2
    assert np.allclose(m, sig ** 2 * (1 + a) * np.exp(-a), rtol=1e-13, atol=0)
    N1 = np.array([[0.0, 0.0, 1.0]])
    N2 = np.array([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [0.0, 0.6, 0.8]])
    nd = uq.covariance("normal_dot", sig, ell, X1, N1, pts[:3], N2)[0]
    assert np.allclose(nd, sig ** 2 * np.array([1.0, 0.0, 0.8]), rtol=0, atol=1e-16)
    assert np.all(uq.covariance("constant", sig, ell, X1, None, pts, None) == sig ** 2)
    # d/d ell: Gaussian K r^2/ell^3 at r = ell is sigma^2 e^{-1/2}/ell
    dg = uq.covariance_dell("gaussian", sig, ell, X1, None, pts[1:2], None)[0, 0]
    assert abs(dg - sig ** 2 * np.exp(-0.5) / ell) < 1e-14 * sig ** 2 / ell
    # Matern-3/2: sigma^2 a^2 e^{-a}/ell, a = sqrt3 r/ell; at r = ell/sqrt3 (a = 1): sigma^2 e^{-1}/ell
    dm = uq.covariance_dell("matern32", sig, ell, X1, None, pts[3:4], None)[0, 0]
    assert abs(dm - sig ** 2 * np.exp(-1.0) / ell) < 1e-14 * sig ** 2 / ell


def test_rcs_db_values():
    """Display transform 10 log10(4 pi V / |p|^2): V = 1/(4 pi) is 0 dB, ten
    times that is 10 dB, |p|^2 = 2 subtracts 10 log10 2, and negative
    combination-technique values are clamped (very low dB, finite)."""
    V = np.array([1.0, 10.0, 1e-3, -1e-9]) / (4.0 * np.pi)
    db = uq.rcs_db(V)
    assert abs(db[0]) < 1e-13 and abs(db[1] - 10.0) < 1e-13 and abs(db[2] + 30.0) < 1e-12
    assert np.isfinite(db[3]) and db[3] < -2900.0
    assert abs(uq.rcs_db(V[:1], pol_norm2=2.0)[0] + 10.0 * np.log10(2.0)) < 1e-13


@pytest.mark.parametrize("kind", ["gaussian", "matern32"])
def test_variance_adjoint_route_equals_sigma_route(oracle_levels, kind):
    """The variance-only route V_r = sum sign mult Re (P1 K P2^H)_rr with
    P_l = FF_l Z_l^{-1} Wgt_l equals the Sigma route angle by angle."""
    xh = workloads.angles_xz(23)
    levels = {s: oracle_levels(s) for s in (0, 1, 2)}
    V, _, _, _, _ = uq.second_moment(None, 1.0, 0, 2, kind, 0.01, 0.5, xh, levels=levels)
    Va = uq.variance_adjoint_route(levels, 0, 2, kind, 0.01, 0.5, xh)
    assert np.abs(Va - V).max() < 1e-11 * np.abs(V).max()


def test_near_field_translation_identity(oracle_levels):
    """Rigid translation c ~ N(0, sigma^2 I) of the sphere: the scattered
    field moves with it, E_c(x) = e^{i k d.c} E(x - c), so
    Var[E'_comp](x) = sigma^2 sum_j |i k d_j E_comp(x) - d_j E_comp(x)|^2
    (d_j: partial derivative, from central differences of the Mie series).
    The discretised near-field variance (K = sigma^2 n(x).n(y), v_n = v_r)
    converges to it at second order (s = 1, 2, 3, k = 1, points at r = 2)."""
    from oracle import mie_shape
    k, d = 1.0, np.array([0.0, 0.0, 1.0])
    g = np.random.default_rng(1).standard_normal((12, 3))
    P = 2.0 * g / np.linalg.norm(g, axis=1, keepdims=True)

    def mie_at(X):
        r = np.linalg.norm(X, axis=1)
        return np.stack([mie_shape.mie_fields(k, ri, np.array([np.arccos(x[2] / ri)]),
                                              np.array([np.arctan2(x[1], x[0])]), part="scattered")[0]
                         for ri, x in zip(r, X)])

    E = mie_at(P)
    h = 1e-4
    ref = np.zeros((len(P), 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        dE = (mie_at(P + e) - mie_at(P - e)) / (2 * h)
        ref += np.abs(1j * k * d[j] * E - dE) ** 2
    errs = []
    for s in (1, 2, 3):
        lv = oracle_levels(s, k, "normal")
        C = uq.rhs_correlation(lv, lv, "normal_dot", 1.0, 1.0)
        NF = efie.near_field_matrix(lv.mesh, k, P)
        V = uq.pair_variance(NF, uq.two_sided_solve(lv, lv, C), NF)
        errs.append(_rel(V.T, ref))
    assert errs[-1] < 2e-2 and errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
