"""Mie series for plane-wave scattering by a perfectly conducting or a
dielectric sphere.

The paper validates its discretisation on the unit sphere against the Mie
series (sphere experiment).  Here the PEC case, written from the textbook
series (Bohren & Huffman, ch. 4) in the limit of infinite refractive index:
    a_n = psi_n'(x) / xi_n'(x),   b_n = psi_n(x) / xi_n(x),   x = k a,
    psi_n = x j_n(x),  xi_n = x h_n^(1)(x),
    S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),
    S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n),
for E^inc = e_x exp(i k z) and time dependence exp(-i w t).  The scattered
field behaves as e^{ikr}/(-ikr) [cos(phi) S2 e_theta - sin(phi) S1 e_phi];
with the paper's normalisation E^sc ~ e^{ikr}/(4 pi r) F this gives
    F = (4 pi / (-i k)) [cos(phi) S2 e_theta - sin(phi) S1 e_phi].

Dielectric sphere (the paper's DE problem, all of its experiments): relative
permittivity eps_r and permeability mu_r inside, refractive index
m = sqrt(eps_r mu_r), the same S1, S2 with (Bohren & Huffman, sec. 4.4)
    a_n = (m^2 j_n(mx) psi_n'(x) - mu_r j_n(x) psi_n'(mx))
          / (m^2 j_n(mx) xi_n'(x) - mu_r h_n(x) psi_n'(mx)),
    b_n = (mu_r j_n(mx) psi_n'(x) - j_n(x) psi_n'(mx))
          / (mu_r j_n(mx) xi_n'(x) - h_n(x) psi_n'(mx)),
psi_n'(rho) the derivative of rho j_n(rho) with respect to its argument.
"""

from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def coefficients(x: float, nmax: int | None = None):
    if nmax is None:
        nmax = int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 12))
    n = np.arange(1, nmax + 1)
    j = spherical_jn(n, x)
    jd = spherical_jn(n, x, derivative=True)
    y = spherical_yn(n, x)
    yd = spherical_yn(n, x, derivative=True)
    h = j + 1j * y
    hd = jd + 1j * yd
    psi = x * j
    dpsi = j + x * jd
    xi = x * h
    dxi = h + x * hd
    return n, dpsi / dxi, psi / xi


def dielectric_coefficients(x: float, eps_r: complex, mu_r: complex = 1.0, nmax: int | None = None):
    """(n, a_n, b_n) of the dielectric sphere, size parameter x = k a."""
    m = np.sqrt(complex(eps_r) * complex(mu_r))
    if nmax is None:
        xm = max(x, abs(m) * x)
        nmax = int(np.ceil(xm + 4.0 * xm ** (1.0 / 3.0) + 12))
    n = np.arange(1, nmax + 1)
    j = spherical_jn(n, x)
    jd = spherical_jn(n, x, derivative=True)
    h = j + 1j * spherical_yn(n, x)
    hd = jd + 1j * spherical_yn(n, x, derivative=True)
    dpsi = j + x * jd
    dxi = h + x * hd
    mx = m * x
    jm = spherical_jn(n, mx)
    dpsim = jm + mx * spherical_jn(n, mx, derivative=True)
    an = (m * m * jm * dpsi - mu_r * j * dpsim) / (m * m * jm * dxi - mu_r * h * dpsim)
    bn = (mu_r * jm * dpsi - j * dpsim) / (mu_r * jm * dxi - h * dpsim)
    return n, an, bn


def _far_field_from_coefficients(k: float, n, an, bn, xh: np.ndarray) -> np.ndarray:
    xh = np.asarray(xh, dtype=np.float64)
    th = np.arccos(np.clip(xh[:, 2], -1.0, 1.0))
    ph = np.arctan2(xh[:, 1], xh[:, 0])
    mu = np.cos(th)
    N = len(n)
    pi = np.zeros((N + 1, len(mu)))
    tau = np.zeros((N + 1, len(mu)))
    pi[1] = 1.0
    for m in range(1, N + 1):
        if m >= 2:
            pi[m] = ((2 * m - 1) / (m - 1)) * mu * pi[m - 1] - (m / (m - 1)) * pi[m - 2]
        tau[m] = m * mu * pi[m] - (m + 1) * pi[m - 1]
    c = ((2 * n + 1) / (n * (n + 1)))[:, None]
    S1 = np.sum(c * (an[:, None] * pi[1:] + bn[:, None] * tau[1:]), axis=0)
    S2 = np.sum(c * (an[:, None] * tau[1:] + bn[:, None] * pi[1:]), axis=0)
    e_th = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], axis=1)
    e_ph = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], axis=1)
    amp = 4.0 * np.pi / (-1j * k)
    return amp * ((np.cos(ph) * S2)[:, None] * e_th - (np.sin(ph) * S1)[:, None] * e_ph)


def pec_far_field(k: float, a: float, xh: np.ndarray, nmax: int | None = None) -> np.ndarray:
    """Far field F (n_a, 3) of the PEC sphere of radius a centred at the
    origin, incident field e_x exp(i k z)."""
    n, an, bn = coefficients(k * a, nmax)
    return _far_field_from_coefficients(k, n, an, bn, xh)


def dielectric_far_field(k: float, a: float, eps_r: complex, mu_r: complex, xh: np.ndarray,
                         nmax: int | None = None) -> np.ndarray:
    """Far field F (n_a, 3) of the dielectric sphere of radius a centred at the
    origin (exterior wavenumber k), incident field e_x exp(i k z)."""
    n, an, bn = dielectric_coefficients(k * a, eps_r, mu_r, nmax)
    return _far_field_from_coefficients(k, n, an, bn, xh)


def pec_far_field_radius_derivative(k: float, a: float, xh: np.ndarray, h: float = 1e-3) -> np.ndarray:
    """d F / d a (breathing mode) by the 5-point central difference of the
    exact series in the radius (truncation error O(h^4))."""
    f = lambda r: pec_far_field(k, r, xh)
    return (-f(a + 2 * h) + 8 * f(a + h) - 8 * f(a - h) + f(a - 2 * h)) / (12 * h)


def extinction_scattering(k: float, a: float):
    """(Q_ext, Q_sca) efficiencies from the series coefficients."""
    x = k * a
    n, an, bn = coefficients(x)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(an + bn))
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(an) ** 2 + np.abs(bn) ** 2))
    return qext, qsca


def dielectric_far_field_oriented(k: float, a: float, eps_r: complex, mu_r: complex, d, p, xh: np.ndarray,
                                  nmax: int | None = None) -> np.ndarray:
    """Far field F (n_a, 3) of the dielectric sphere for the plane wave
    p exp(i k d.x) (real unit p orthogonal to the unit d): the series of
    dielectric_far_field in the frame e1 = p, e2 = d x p, e3 = d, where the
    incidence is e1 exp(i k x3), rotated back."""
    d = np.asarray(d, dtype=np.float64)
    e1 = np.asarray(p, dtype=np.float64)
    e3 = d / np.linalg.norm(d)
    e1 = e1 / np.linalg.norm(e1)
    e2 = np.cross(e3, e1)
    Rm = np.stack([e1, e2, e3])                       # rows: the frame's axes
    xl = np.asarray(xh, dtype=np.float64) @ Rm.T      # directions in the frame
    return dielectric_far_field(k, a, eps_r, mu_r, xl, nmax) @ Rm
