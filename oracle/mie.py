"""Mie series for a perfectly conducting sphere.

Test infrastructure only. The paper's primary reference for the sphere is
the analytical Mie series solution (Section 2.2). We use the Bohren &
Huffman (1983) form with the PEC limit of the coefficients,

    a_n = psi_n'(x) / xi_n'(x),   b_n = psi_n(x) / xi_n(x),   x = k a,

with Riccati-Bessel psi_n(x) = x j_n(x), xi_n(x) = x h_n^(1)(x), the angle
functions pi_n, tau_n by upward recurrence, and the series truncated at
n_max = ceil(x + 4.05 x^(1/3) + 2) (Wiscombe 1980). For a unit x-polarised
wave along +z, sigma_tt = (4 pi / k^2) |S2(Theta)|^2 cos^2(phi). Our wave
travels toward -z, so the scattering angle is Theta = pi - theta.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def n_terms(x: float) -> int:
    return int(math.ceil(x + 4.05 * x ** (1.0 / 3.0) + 2.0))


def coefficients(x: float, nmax: int | None = None):
    nmax = n_terms(x) if nmax is None else nmax
    n = np.arange(1, nmax + 1)
    jn = spherical_jn(n, x)
    jnp = spherical_jn(n, x, derivative=True)
    yn = spherical_yn(n, x)
    ynp = spherical_yn(n, x, derivative=True)
    psi = x * jn
    dpsi = jn + x * jnp
    xi = x * (jn + 1j * yn)
    dxi = (jn + 1j * yn) + x * (jnp + 1j * ynp)
    return n, dpsi / dxi, psi / xi


def amplitudes(x: float, Theta: np.ndarray):
    """S1(Theta), S2(Theta)."""
    n, a, b = coefficients(x)
    mu = np.cos(np.asarray(Theta, dtype=np.float64))
    pi_prev = np.zeros_like(mu)
    pi_cur = np.ones_like(mu)
    S1 = np.zeros(mu.shape, dtype=np.complex128)
    S2 = np.zeros(mu.shape, dtype=np.complex128)
    for idx, nn in enumerate(n):
        if nn == 1:
            pi_n = np.ones_like(mu)
        else:
            pi_n = ((2 * nn - 1) / (nn - 1)) * mu * pi_cur - (nn / (nn - 1)) * pi_prev
        if nn > 1:
            pi_prev, pi_cur = pi_cur, pi_n
        else:
            pi_prev, pi_cur = np.zeros_like(mu), pi_n
        tau_n = nn * mu * pi_n - (nn + 1) * pi_prev
        c = (2 * nn + 1) / (nn * (nn + 1))
        S1 += c * (a[idx] * pi_n + b[idx] * tau_n)
        S2 += c * (a[idx] * tau_n + b[idx] * pi_n)
    return S1, S2


def sigma_tt(k: float, radius: float, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """sigma_tt on the (theta, phi) grid for the x-polarised wave toward -z."""
    _, S2 = amplitudes(k * radius, math.pi - np.asarray(theta))
    return (4 * math.pi / k**2) * np.abs(S2)[:, None] ** 2 * np.cos(np.asarray(phi))[None, :] ** 2


def efficiencies(x: float):
    """(Q_ext, Q_sca) from the coefficients."""
    n, a, b = coefficients(x)
    qext = (2.0 / x**2) * np.sum((2 * n + 1) * np.real(a + b))
    qsca = (2.0 / x**2) * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return float(qext), float(qsca)
