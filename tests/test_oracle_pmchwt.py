"""Pins of the dielectric oracle (oracle/pmchwt.py, oracle/mie.py): the
dielectric Mie series against its closed-form limits, and the Galerkin PMCHWT
system against the Mie series, the extinction of a sphere with the exterior's
material, a direct evaluation of the MFIO local blocks and the rank-one
second-moment identity of the sphere experiment."""

import numpy as np
import pytest

import workloads
from oracle import efie, mie, pmchwt
from oracle import mesh as meshmod

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

K0, EPS, MU = 3.0, 2.1, 1.0          # the sphere experiment's material and exterior wavenumber
D, P = [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# ----------------------------------------------------------------------------- Mie series
def test_mie_no_contrast_is_zero():
    n, a, b = mie.dielectric_coefficients(2.0, 1.0, 1.0)
    assert np.abs(a).max() < 1e-15 and np.abs(b).max() < 1e-15


def test_mie_lossless_coefficients_on_circle():
    """Real m, mu_r: energy conservation per multipole, Re a = |a|^2, Re b = |b|^2."""
    for er, mr in ((2.1, 1.0), (4.0, 2.5)):
        n, a, b = mie.dielectric_coefficients(3.0, er, mr)
        assert np.abs(a.real - np.abs(a) ** 2).max() < 1e-13
        assert np.abs(b.real - np.abs(b) ** 2).max() < 1e-13


def test_mie_duality_swaps_coefficients():
    """Exchanging eps_r and mu_r exchanges the electric and magnetic multipoles."""
    n, a1, b1 = mie.dielectric_coefficients(2.0, 3.0, 2.0, nmax=20)
    n, a2, b2 = mie.dielectric_coefficients(2.0, 2.0, 3.0, nmax=20)
    assert np.abs(a1 - b2).max() < 1e-14 and np.abs(b1 - a2).max() < 1e-14


def test_mie_rayleigh_limit():
    """a_1 -> -(2i/3) x^3 (m^2 - 1)/(m^2 + 2) for a small non-magnetic sphere."""
    x, er = 1e-3, 2.1
    n, a, b = mie.dielectric_coefficients(x, er, 1.0, nmax=3)
    ref = -2j / 3 * x ** 3 * (er - 1) / (er + 2)
    assert abs(a[0] / ref - 1) < 1e-6


def test_mie_pec_limit():
    """A large complex index tends to the perfect conductor at rate 1/|m|."""
    n, ap, bp = mie.coefficients(2.0, 12)
    errs = []
    for s in (50, 100, 200):
        n, ad, bd = mie.dielectric_coefficients(2.0, (s * (1 + 1j)) ** 2, 1.0, nmax=12)
        errs.append(max(np.abs(ad - ap).max(), np.abs(bd - bp).max()))
    assert errs[-1] < 5e-3 and 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


# ----------------------------------------------------------------------------- PMCHWT
@pytest.fixture(scope="module")
def sphere_meshes():
    return {s: meshmod.build(*workloads.icosphere(s)) for s in (1, 2)}


@pytest.fixture(scope="module")
def solves(sphere_meshes):
    return {s: pmchwt.solve(sphere_meshes[s], K0, EPS, MU, D, P) for s in (1, 2)}


def test_pmchwt_converges_to_mie(sphere_meshes, solves):
    """The far field of the Galerkin PMCHWT solution approaches the Mie series
    at second order in h (the paper's sphere experiment setting: eps_r 2.1,
    k0 3, d = e_x, p = e_z); the paper reports O(h^2) for the first moment."""
    xh = workloads.angles_xy(91)
    Fm = mie.dielectric_far_field_oriented(K0, 1.0, EPS, MU, D, P, xh)
    e = [_rel(pmchwt.far_field(sphere_meshes[s], K0, solves[s][2], xh), Fm) for s in (1, 2)]
    print(f"PMCHWT vs Mie: s=1 {e[0]:.3e}, s=2 {e[1]:.3e}, rate {e[0] / e[1]:.2f}")
    assert e[1] < 0.06 and e[0] / e[1] > 3.0


def test_pmchwt_extinction_without_contrast(sphere_meshes):
    """eps_r = mu_r = 1: the traces of the incident field solve the continuous
    equations and radiate nothing outside, so the discrete far field vanishes
    with the mesh (faster than the field itself converges)."""
    xh = workloads.angles_xy(37)
    F = []
    for s in (1, 2):
        Z, b, u = pmchwt.solve(sphere_meshes[s], K0, 1.0, 1.0, D, P)
        F.append(np.linalg.norm(pmchwt.far_field(sphere_meshes[s], K0, u, xh)))
    # scale: the incident traces' own far field, radiated by J alone
    J = np.linalg.solve(efie.assemble(sphere_meshes[2], K0), -efie.incident_rhs(sphere_meshes[2], K0, D, P))
    scale = np.linalg.norm(efie.far_field(sphere_meshes[2], K0, J, xh))
    print(f"extinction: |F| s=1 {F[0]:.3e}, s=2 {F[1]:.3e} (scale {scale:.3e})")
    assert F[1] < 2e-3 * scale and F[0] / F[1] > 5.0


def test_mfio_local_blocks_direct(sphere_meshes):
    """The vectorised MFIO blocks against the integrand written out point pair
    by point pair as a determinant, det[phi_a(x), grad G, phi_b(y)]."""
    m = sphere_meshes[1]
    bq = efie.basis_at_points(m)
    X, W, Phi, _ = bq
    I = np.array([0, 3, 17, 40])
    J = np.array([60, 79, 5, 11])
    blk = pmchwt.local_regular_k(m, K0, I, J, bq)
    for p, (i, j) in enumerate(zip(I, J)):
        ref = np.zeros((3, 3), dtype=complex)
        for a in range(3):
            for b in range(3):
                for q1 in range(6):
                    for q2 in range(6):
                        d = X[i, q1] - X[j, q2]
                        R = np.linalg.norm(d)
                        g = (1j * K0 * R - 1) * np.exp(1j * K0 * R) / (4 * np.pi * R ** 3)
                        ref[a, b] += W[i, q1] * W[j, q2] * g * np.linalg.det(
                            np.stack([Phi[i, a, q1], d, Phi[j, b, q2]]).astype(complex))
        assert np.abs(blk[p] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_mfio_matrix_symmetric(sphere_meshes):
    """grad_y G = -grad_x G makes the MFIO Galerkin matrix symmetric: exactly
    (to rounding) on regular pairs, to quadrature accuracy on touching ones."""
    m = sphere_meshes[1]
    Kk = pmchwt.assemble_k(m, K0)
    asym = np.linalg.norm(Kk - Kk.T) / np.linalg.norm(Kk)
    print(f"MFIO asymmetry {asym:.2e}")
    assert asym < 1e-6


def test_rank_one_second_moment_identity(sphere_meshes, solves):
    """M2[f] = f (x) f gives M2[xi] = xi (x) xi (sphere experiment): every CT
    block is u_l1 u_l2^H, and the CT far-field second moment of the pair set
    with one level pair equals |F|^2 of that level."""
    xh = workloads.angles_xy(37)
    V, blocks, lev = pmchwt.rank_one_second_moment(sphere_meshes, 1, 2, K0, EPS, MU, D, P, xh, systems=solves)
    for (l1, l2), S in blocks.items():
        ref = np.outer(lev[l1][2], lev[l2][2].conj())
        assert _rel(S, ref) < 1e-12
    V22, _, lev2 = pmchwt.rank_one_second_moment(sphere_meshes, 2, 2, K0, EPS, MU, D, P, xh, systems=solves)
    F2 = pmchwt.far_field(sphere_meshes[2], K0, lev2[2][2], xh)
    assert _rel(V22, np.abs(F2.T) ** 2) < 1e-12
    # the combination of levels 1 and 2 approximates |F_Mie|^2 about as well as level 2 alone
    Fm = mie.dielectric_far_field_oriented(K0, 1.0, EPS, MU, D, P, xh)
    e_ct, e_2 = _rel(V[2], np.abs(Fm[:, 2]) ** 2), _rel(V22[2], np.abs(Fm[:, 2]) ** 2)
    print(f"|F_z|^2 vs Mie: CT(1,2) {e_ct:.3e}, level 2 {e_2:.3e}")
    assert e_ct < 3 * e_2 + 0.05
