"""Mie series for a perfectly conducting sphere (the analytic comparison of
the bistatic sphere experiment, Sec. V.C.1).

Textbook form (Bohren & Huffman 1983, Ch. 4, PEC limit; Ruck et al. 1970):
with x = k a, Riccati-Bessel psi_n(x) = x j_n(x) and xi_n(x) = x h_n^(1)(x),
  a_n = psi_n'(x) / xi_n'(x),   b_n = psi_n(x) / xi_n(x),
  S1(t) = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),
  S2(t) = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n),
with pi_n = P_n^1(cos t)/sin t and tau_n = d P_n^1(cos t)/dt.  Bistatic
sigma = (4 pi / k^2) |S|^2 at scattering angle t from the forward direction;
S2 is the E-plane (co-polar theta component), S1 the H-plane.  Backscatter
(t = pi):  sigma / (pi a^2) = x^-2 |sum (2n+1)(-1)^n (a_n - b_n)|^2.
"""

import math

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def _nmax(x):
    return int(math.ceil(x + 4.05 * x ** (1.0 / 3.0) + 10))


def coefficients(x, nmax=None):
    nmax = nmax or _nmax(x)
    n = np.arange(1, nmax + 1)
    jn = spherical_jn(n, x)
    yn = spherical_yn(n, x)
    jnp = spherical_jn(n, x, derivative=True)
    ynp = spherical_yn(n, x, derivative=True)
    hn = jn + 1j * yn
    hnp = jnp + 1j * ynp
    psi = x * jn
    xi = x * hn
    dpsi = jn + x * jnp
    dxi = hn + x * hnp
    return n, dpsi / dxi, psi / xi


def angular(nmax, theta):
    """pi_n, tau_n for n = 1..nmax at angles theta (upward recurrence)."""
    mu = np.cos(theta)
    pi = np.zeros((nmax + 1,) + np.shape(theta))
    tau = np.zeros_like(pi)
    pi[1] = 1.0
    if nmax >= 2:
        pi[2] = 3.0 * mu
    for n in range(3, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
    for n in range(1, nmax + 1):
        tau[n] = n * mu * pi[n] - (n + 1) * (pi[n - 1] if n >= 1 else 0.0)
    return pi[1:], tau[1:]


def amplitudes(x, theta):
    n, an, bn = coefficients(x)
    pi, tau = angular(len(n), np.asarray(theta, dtype=np.float64))
    c = ((2 * n + 1) / (n * (n + 1)))
    shp = (-1,) + (1,) * np.ndim(theta)
    S1 = np.sum((c * an).reshape(shp) * pi + (c * bn).reshape(shp) * tau, axis=0)
    S2 = np.sum((c * an).reshape(shp) * tau + (c * bn).reshape(shp) * pi, axis=0)
    return S1, S2


def backscatter_efficiency(x):
    """sigma_back / (pi a^2)."""
    n, an, bn = coefficients(x)
    s = np.sum((2 * n + 1) * (-1.0) ** n * (an - bn))
    return abs(s) ** 2 / x ** 2


def backscatter_rcs(radius, k):
    return backscatter_efficiency(k * radius) * math.pi * radius ** 2


def bistatic_rcs(radius, k, scat_angle, plane="E"):
    """sigma (m^2) at scattering angles measured from the forward direction."""
    S1, S2 = amplitudes(k * radius, scat_angle)
    S = S2 if plane == "E" else S1
    return 4.0 * math.pi / k ** 2 * np.abs(S) ** 2


def efficiencies(x):
    """(Q_ext, Q_sca) from the series; equal for a lossless (PEC) sphere."""
    n, an, bn = coefficients(x)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(an + bn))
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(an) ** 2 + np.abs(bn) ** 2))
    return qext, qsca
