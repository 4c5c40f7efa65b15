"""Mesh-free reference for the far-field variance of the shape derivative of
the PEC unit sphere under an isotropic Gaussian perturbation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The sphere experiment of the paper checks the discretisation against the
Mie series.  Here the same is done for the second moment of the shape
derivative, with no mesh at all:

1. Exact fields.  The total field of the plane wave p exp(i k d.x),
   p = e_x, d = e_z, scattered by the PEC unit sphere and its radial
   derivative on r = 1, from the Mie expansion in vector spherical wave
   functions (Bohren & Huffman, ch. 4; PEC coefficients as in mie.py).
2. Boundary data of the shape derivative.  Moving the surface by v n
   (v real, n the outer normal) and differentiating n_t x E_t = 0 at t = 0
   with the normal's derivative -grad_G v and E = E_r n on the surface gives
       n x E' = E_r grad_G v x n - v n x d_r E        (on r = 1),
   written here directly from that derivation (it equals the Hadamard form
   the paper states for the shape-derivative data, but is not taken from it).
3. Exterior problem.  E' is the radiating Maxwell field with that tangential
   trace.  On the sphere the problem is diagonal in vector spherical
   harmonics: with M_lm = h_l(kr) grad_G Y_lm x rhat and
   N_lm = curl M_lm / k,
       rhat x M_lm = h_l(k) grad_G Y_lm,
       rhat x N_lm = [(rho h_l)'/rho](k) rhat x grad_G Y_lm      (r = 1),
   so projecting n x E' on grad_G Y_lm and rhat x grad_G Y_lm (each of
   squared norm l(l+1)) gives the coefficients, and h_l(rho) ~
   (-i)^{l+1} e^{i rho}/rho gives the far field in the normalisation
   E ~ e^{ik|x|}/(4 pi |x|) F.
4. Covariance.  On the unit sphere the chord distance gives
   |x - y|^2 = 2 - 2 x.y, so the Gaussian covariance is a function of x.y
   and (Funk-Hecke / addition theorem)
       K(x, y) = sum_n kappa_n sum_m Y_nm(x) conj Y_nm(y),
       kappa_n = 2 pi int_{-1}^{1} K(t) P_n(t) dt.
   For v with that covariance, Var[F'_c(x)] = sum_n kappa_n sum_m |F'_c[Y_nm](x)|^2.

Every truncation converges exponentially, so the result is exact to
rounding once the degrees are large enough; the discretised variance must
converge to it as the mesh is refined.
"""

from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y, spherical_in, spherical_jn, spherical_yn

from . import mie


# ----------------------------------------------------------------------------- radial functions
def _sph(kind: str, n: np.ndarray, rho: float):
    """z_n(rho) and z_n'(rho) for z = j ('j') or h^(1) ('h')."""
    j, jd = spherical_jn(n, rho), spherical_jn(n, rho, derivative=True)
    if kind == "j":
        return j, jd
    y, yd = spherical_yn(n, rho), spherical_yn(n, rho, derivative=True)
    return j + 1j * y, jd + 1j * yd


def _radial(kind: str, n: np.ndarray, rho: float):
    """The three radial factors of the wave functions, f1 = z_n,
    f2 = (rho z_n)'/rho, f3 = z_n/rho, and their rho-derivatives (from the
    spherical Bessel equation z'' = -(2/rho) z' - (1 - n(n+1)/rho^2) z)."""
    z, zd = _sph(kind, n, rho)
    zdd = -(2.0 / rho) * zd - (1.0 - n * (n + 1) / rho ** 2) * z
    f1, d1 = z, zd
    f2 = z / rho + zd
    d2 = -z / rho ** 2 + zd / rho + zdd
    f3 = z / rho
    d3 = zd / rho - z / rho ** 2
    return (f1, f2, f3), (d1, d2, d3)


def _pi_tau(nmax: int, mu: np.ndarray):
    """Angular functions pi_n, tau_n (n = 1..nmax) of the m = 1 wave functions."""
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros((nmax + 1,) + mu.shape)
    pi[1] = 1.0
    for n in range(1, nmax + 1):
        if n >= 2:
            pi[n] = ((2 * n - 1) / (n - 1)) * mu * pi[n - 1] - (n / (n - 1)) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def _frames(th, ph):
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    er = np.stack([st * cp, st * sp, ct], -1)
    et = np.stack([ct * cp, ct * sp, -st], -1)
    ep = np.stack([-sp, cp, np.zeros_like(th)], -1)
    return er, et, ep


def mie_fields(k: float, r: float, th: np.ndarray, ph: np.ndarray, nmax: int | None = None,
               part: str = "total", derivative: bool = False) -> np.ndarray:
    """Incident, scattered or total field (..., 3) (Cartesian components) of
    the plane wave e_x exp(i k z) and the PEC unit sphere at radius r and
    angles (th, ph), or its radial derivative d/dr.  Series (Bohren & Huffman,
    ch. 4):  E_inc = sum E_n (M1_o1n - i N1_e1n),
    E_sca = sum E_n (i a_n N3_e1n - b_n M3_o1n),  E_n = i^n (2n+1)/(n(n+1))."""
    rho = k * r
    n, an, bn = mie.coefficients(k * 1.0, nmax)
    nmax = len(n)
    En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
    pi, tau = _pi_tau(nmax, np.cos(th))
    st = np.sin(th)
    cp, sp = np.cos(ph), np.sin(ph)
    er, et, ep = _frames(th, ph)
    out = np.zeros(th.shape + (3,), dtype=np.complex128)
    terms = []
    if part in ("incident", "total"):
        terms.append(("j", En, -1j * En))          # coefficient of M_o1n, of N_e1n
    if part in ("scattered", "total"):
        terms.append(("h", -bn * En, 1j * an * En))
    for kind, cM, cN in terms:
        f, df = _radial(kind, n, rho)
        if derivative:                               # d/dr = k d/drho
            f = tuple(k * x for x in df)
        f1, f2, f3 = (x[:, None] if np.ndim(th) == 1 else x.reshape((-1,) + (1,) * np.ndim(th)) for x in f)
        cMb = cM.reshape((-1,) + (1,) * np.ndim(th))
        cNb = cN.reshape((-1,) + (1,) * np.ndim(th))
        nn = (n * (n + 1)).reshape((-1,) + (1,) * np.ndim(th))
        # M_o1n = cos(ph) pi z e_th - sin(ph) tau z e_ph
        # N_e1n = cos(ph) n(n+1) sin(th) pi z/rho e_r + cos(ph) tau (rho z)'/rho e_th
        #         - sin(ph) pi (rho z)'/rho e_ph
        Mth = np.sum(cMb * cp * pi * f1, 0)
        Mph = np.sum(cMb * (-sp) * tau * f1, 0)
        Nr = np.sum(cNb * cp * nn * st * pi * f3, 0)
        Nth = np.sum(cNb * cp * tau * f2, 0)
        Nph = np.sum(cNb * (-sp) * pi * f2, 0)
        out += (Nr[..., None] * er + (Mth + Nth)[..., None] * et + (Mph + Nph)[..., None] * ep)
    return out


# ----------------------------------------------------------------------------- harmonics
def _y(l: int, mu: int, th: np.ndarray) -> np.ndarray:
    """y_l^mu(th) = Y_l^mu(th, 0) (real): Y_l^mu(th, ph) = y_l^mu(th) e^{i mu ph}
    (orthonormal complex harmonics, Condon-Shortley phase); 0 for |mu| > l."""
    if abs(mu) > l:
        return np.zeros(np.shape(th))
    return np.real(sph_harm_y(l, mu, th, 0.0))


def _dy(l: int, mu: int, th: np.ndarray) -> np.ndarray:
    """d y_l^mu / d th = mu cot(th) y_l^mu + sqrt((l-mu)(l+mu+1)) y_l^{mu+1}."""
    if abs(mu) > l:
        return np.zeros(np.shape(th))
    return mu / np.tan(th) * _y(l, mu, th) + np.sqrt((l - mu) * (l + mu + 1.0)) * _y(l, mu + 1, th)


def surface_grad_Y(l: int, m: int, th: np.ndarray, ph: np.ndarray):
    """Y_lm and grad_G Y_lm (Cartesian, (..., 3)) on the unit sphere."""
    e = np.exp(1j * m * ph)
    Y = _y(l, m, th) * e
    _, et, ep = _frames(th, ph)
    G = (_dy(l, m, th) * e)[..., None] * et + (1j * m * _y(l, m, th) / np.sin(th) * e)[..., None] * ep
    return Y, G


# ----------------------------------------------------------------------------- exterior problem
class SphereGrid:
    """Gauss-Legendre in cos(th) x uniform ph product rule on the unit sphere
    (points th[j], ph[q]; weight w[j] * 2 pi / n_ph)."""

    def __init__(self, n_th: int, n_ph: int):
        x, w = np.polynomial.legendre.leggauss(n_th)
        self.th = np.arccos(x)
        self.w = w
        self.n_ph = n_ph
        self.ph = 2.0 * np.pi * np.arange(n_ph) / n_ph
        self.TH, self.PH = np.meshgrid(self.th, self.ph, indexing="ij")
        self._cache = {}

    def y_dy(self, l: int, mu: int):
        """y_l^mu and its th-derivative at the grid's th nodes (cached)."""
        key = (l, mu)
        if key not in self._cache:
            self._cache[key] = (_y(l, mu, self.th), _dy(l, mu, self.th))
        return self._cache[key]

    def local(self, E: np.ndarray):
        """(r, th, ph) components of a Cartesian field (n_th, n_ph, 3) on the grid."""
        er, et, ep = _frames(self.TH, self.PH)
        return np.sum(E * er, -1), np.sum(E * et, -1), np.sum(E * ep, -1)

    def azimuthal(self, f: np.ndarray, mu: int) -> np.ndarray:
        """(2 pi / n_ph) sum_q f(th_j, ph_q) e^{-i mu ph_q}  for every th_j."""
        return (2.0 * np.pi / self.n_ph) * np.fft.fft(f, axis=1)[:, mu % self.n_ph]


def _output_points(xh: np.ndarray, eps: float = 1e-6):
    """Angles of the output directions; a direction within eps of a pole is
    replaced by the two points at polar distance eps on either side of it
    along its meridian (their mean gives the pole value to O(eps^2))."""
    xh = np.asarray(xh, dtype=np.float64)
    th = np.arccos(np.clip(xh[:, 2], -1.0, 1.0))
    ph = np.arctan2(xh[:, 1], xh[:, 0])
    th = np.clip(th, eps, np.pi - eps)
    th2 = np.concatenate([th, th])
    ph2 = np.concatenate([ph, ph + np.pi])
    near = np.sin(np.arccos(np.clip(xh[:, 2], -1.0, 1.0))) < eps
    return th2, ph2, near


def _combine(F2: np.ndarray, near: np.ndarray) -> np.ndarray:
    n = len(near)
    F = F2[:n].copy()
    F[near] = 0.5 * (F2[:n][near] + F2[n:][near])
    return F


def far_field_from_trace(k: float, grid: SphereGrid, g_th: np.ndarray, g_ph: np.ndarray, orders, lmax: int,
                         th_o: np.ndarray, ph_o: np.ndarray, out_cache: dict | None = None) -> np.ndarray:
    """Far field (n_out, 3) at angles (th_o, ph_o) of the radiating Maxwell
    field E outside the unit sphere with rhat x E = g on r = 1 (g given by its
    th and ph components on the grid), keeping vector harmonics of degree
    1..lmax and the listed azimuthal orders:
        alpha_l = <g, grad_G Y_l^mu> / l(l+1),  beta_l = <g, rhat x grad_G Y_l^mu> / l(l+1),
        E = sum alpha_l/h_l(k) M_l^mu + beta_l k/(rho h_l)'(k) N_l^mu."""
    er, et, ep = _frames(th_o, ph_o)
    st = np.sin(grid.th)
    F = np.zeros(th_o.shape + (3,), dtype=np.complex128)
    for mu in orders:
        gt = grid.azimuthal(g_th, mu)
        gp = grid.azimuthal(g_ph, mu)
        e_o = np.exp(1j * mu * ph_o)
        for l in range(max(1, abs(mu)), lmax + 1):
            y, dy = grid.y_dy(l, mu)
            ll = l * (l + 1.0)
            alpha = np.sum(grid.w * (gt * dy - gp * 1j * mu * y / st)) / ll
            beta = np.sum(grid.w * (gt * 1j * mu * y / st + gp * dy)) / ll
            h, hd = _sph("h", np.array([l]), k)
            a = alpha / h[0]
            b = beta / (h[0] / k + hd[0])
            if out_cache is not None and (l, mu) in out_cache:
                yo, dyo = out_cache[(l, mu)]
            else:
                yo, dyo = _y(l, mu, th_o), _dy(l, mu, th_o)
                if out_cache is not None:
                    out_cache[(l, mu)] = (yo, dyo)
            G = (dyo * e_o)[:, None] * et + (1j * mu * yo / np.sin(th_o) * e_o)[:, None] * ep
            C = (dyo * e_o)[:, None] * ep - (1j * mu * yo / np.sin(th_o) * e_o)[:, None] * et
            F += (4.0 * np.pi / k) * (-a * (-1j) ** (l + 1) * C + b * (-1j) ** l * G)
    return F


def shape_derivative_trace(grid: SphereGrid, Er, dEt, dEp, l: int, m: int):
    """(th, ph) components of rhat x E' = E_r grad_G v x rhat - v rhat x d_r E
    for v = Y_l^m:  g_th = E_r v_ph + v dE_ph,  g_ph = -E_r v_th - v dE_th."""
    e = np.exp(1j * m * grid.ph)[None, :]
    y, dy = grid.y_dy(l, m)
    v = y[:, None] * e
    v_th = dy[:, None] * e
    v_ph = (1j * m * y / np.sin(grid.th))[:, None] * e
    return Er * v_ph + v * dEp, -Er * v_th - v * dEt


class SphereShapeDerivative:
    """F'[Y_l^m] of the PEC unit sphere under the plane wave e_x exp(i k z)."""

    def __init__(self, k: float, l_v: int, n_grid: int | None = None):
        self.k = k
        n_e = len(mie.coefficients(k)[0])
        self.lmax = l_v + n_e + 2
        ng = n_grid or (self.lmax + 10)
        self.grid = SphereGrid(ng, 2 * self.lmax + 8)
        g = self.grid
        self._out_key = None
        self._out_cache = {}
        self.Er, _, _ = g.local(mie_fields(k, 1.0, g.TH, g.PH))
        _, self.dEt, self.dEp = g.local(mie_fields(k, 1.0, g.TH, g.PH, derivative=True))

    def far_field(self, l: int, m: int, xh: np.ndarray) -> np.ndarray:
        th2, ph2, near = _output_points(xh)
        key = np.asarray(xh, dtype=np.float64).tobytes()
        if key != self._out_key:           # harmonics at the output angles, cached per angle set
            self._out_key, self._out_cache = key, {}
        gt, gp = shape_derivative_trace(self.grid, self.Er, self.dEt, self.dEp, l, m)
        F2 = far_field_from_trace(self.k, self.grid, gt, gp, (m - 1, m + 1), self.lmax, th2, ph2,
                                  self._out_cache)
        return _combine(F2, near)


def scattered_far_field_from_trace(k: float, xh: np.ndarray) -> np.ndarray:
    """Far field of the Mie scattered field recomputed from its tangential
    trace on r = 1 through far_field_from_trace (a check of the exterior
    solver against the series far field of mie.py)."""
    n_e = len(mie.coefficients(k)[0])
    lmax = n_e + 4
    grid = SphereGrid(lmax + 10, 2 * lmax + 8)
    _, Et, Ep = grid.local(mie_fields(k, 1.0, grid.TH, grid.PH, part="scattered"))
    th2, ph2, near = _output_points(xh)
    # rhat x E = E_th e_ph - E_ph e_th
    F2 = far_field_from_trace(k, grid, -Ep, Et, (-1, 1), lmax, th2, ph2)
    return _combine(F2, near)


def gaussian_kappa(sigma: float, ell: float, nmax: int) -> np.ndarray:
    """kappa_n = 2 pi int_{-1}^{1} K(t) P_n(t) dt for the Gaussian covariance
    sigma^2 exp(-|x-y|^2/(2 ell^2)) with |x-y|^2 = 2 - 2t on the unit sphere:
    K(t) = sigma^2 e^{-a} e^{a t}, a = 1/ell^2, and int e^{a t} P_n(t) dt =
    2 i_n(a) (modified spherical Bessel function), so
    kappa_n = 4 pi sigma^2 e^{-a} i_n(a)."""
    a = 1.0 / ell ** 2
    n = np.arange(nmax + 1)
    return 4.0 * np.pi * sigma ** 2 * np.exp(-a) * spherical_in(n, a)


def variance_gaussian(k: float, sigma: float, ell: float, xh: np.ndarray, n_cov: int | None = None,
                      rel_cut: float = 1e-15) -> np.ndarray:
    """Var[F'_c](xh) (3, n_a) for the radial Gaussian perturbation of the PEC
    unit sphere (incidence e_x exp(i k z)):  sum_n kappa_n sum_m |F'_c[Y_n^m]|^2,
    truncated at covariance degree n_cov (default: the last n with
    (2n+1) kappa_n above rel_cut times the leading term)."""
    kap = gaussian_kappa(sigma, ell, 120)
    if n_cov is None:
        tot = (2 * np.arange(121) + 1) * np.abs(kap)
        n_cov = int(np.nonzero(tot > rel_cut * tot.max())[0].max())
    kap = kap[: n_cov + 1]
    sd = SphereShapeDerivative(k, n_cov)
    V = np.zeros((len(xh), 3))
    for n in range(n_cov + 1):
        for m in range(-n, n + 1):
            V += kap[n] * np.abs(sd.far_field(n, m, xh)) ** 2
    return V.T
