"""Closed-form surface integrals of 1/R and (r' - rho)/R over a flat triangle.

The EFIE kernel of eqs. (2)-(3) is singular when the observation and source
triangles touch.  The standard treatment (Wilton et al., IEEE TAP 1984;
Graglia, IEEE TAP 1993) removes the 1/R part of G and integrates it in closed
form over the source triangle; the remainder (exp(-jkR) - 1)/R is bounded and
is integrated numerically.  For an observation point r, with n the unit normal
of the source triangle, d = n.(r - v0) its height above the plane and rho its
projection, each edge i (from p_a to p_b, counter-clockwise) has the unit
direction s_i, the outward in-plane normal u_i = s_i x n, the tangential
coordinates l+- = (p_b|p_a - rho).s_i, the signed distance t0 = (p_a - rho).u_i,
R0^2 = t0^2 + d^2 and R+- = sqrt(l+-^2 + R0^2).  Then

  int 1/R dS'            = sum_i [ t0 F_i - |d| (atan(t0 l+ / (R0^2 + |d| R+))
                                                - atan(t0 l- / (R0^2 + |d| R-))) ]
  int (r' - rho)/R dS'   = 1/2 sum_i u_i [ R0^2 F_i + l+ R+ - l- R- ]

with F_i = ln((R+ + l+) / (R- + l-)).
"""

import numpy as np


def _dot(a, b):
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def triangle_potentials(r, tv):
    """r: (K, 3) points; tv: (K, 3, 3) triangle vertices (CCW).

    Returns (I1, Irho, rho): int 1/R dS' (K,), int (r' - rho)/R dS' (K, 3) and
    the projection rho (K, 3) of r onto the triangle's plane.
    """
    r = np.asarray(r, dtype=np.float64)
    v0, v1, v2 = tv[:, 0], tv[:, 1], tv[:, 2]
    n = np.cross(v1 - v0, v2 - v0)
    n = n / np.sqrt(_dot(n, n))[:, None]
    d = _dot(r - v0, n)
    rho = r - d[:, None] * n
    ad = np.abs(d)
    I1 = np.zeros(len(r))
    Irho = np.zeros((len(r), 3))
    verts = (v0, v1, v2)
    for e in range(3):
        pa, pb = verts[e], verts[(e + 1) % 3]
        L = pb - pa
        s = L / np.sqrt(_dot(L, L))[:, None]
        u = np.cross(s, n)
        lp = _dot(pb - rho, s)
        lm = _dot(pa - rho, s)
        t0 = _dot(pa - rho, u)
        R0sq = t0 * t0 + d * d
        Rp = np.sqrt(lp * lp + R0sq)
        Rm = np.sqrt(lm * lm + R0sq)
        # ln((R+ + l+)/(R- + l-)) == ln((R- - l-)/(R+ - l+)); use the form
        # whose arguments do not cancel.
        with np.errstate(divide="ignore", invalid="ignore"):
            F = np.where(lp + lm >= 0.0,
                         np.log((Rp + lp) / (Rm + lm)),
                         np.log((Rm - lm) / (Rp - lp)))
            F = np.where(R0sq > 0.0, F, 0.0)
            den_p = R0sq + ad * Rp
            den_m = R0sq + ad * Rm
            beta = np.where(den_p > 0.0, np.arctan(t0 * lp / np.where(den_p > 0, den_p, 1.0)), 0.0) \
                - np.where(den_m > 0.0, np.arctan(t0 * lm / np.where(den_m > 0, den_m, 1.0)), 0.0)
        I1 += t0 * F - ad * beta
        Irho += 0.5 * u * (R0sq * F + lp * Rp - lm * Rm)[:, None]
    return I1, Irho, rho


def triangle_gradient_potential(r, tv):
    """int_T (r - r') / R^3 dS' (K, 3) for points r (K, 3) and triangles tv.

    With rho, d and the per-edge quantities above, the in-plane part is the
    surface divergence theorem applied to grad'_s (1/R) = (rho - r') / R^3,
    sum_i u_i F_i, and the normal part is d int 1/R^3 dS' = sign(d) times the
    solid-angle sum of the same arctangent terms (Graglia, IEEE TAP 1993):

      int (r - r')/R^3 dS' = sum_i u_i F_i + n sign(d) sum_i beta_i,
      beta_i = atan(t0 l+ / (R0^2 + |d| R+)) - atan(t0 l- / (R0^2 + |d| R-)).

    This is the static part of the MFIE kernel (see ``mfie``).  Points on the
    plane of T outside its closure get a zero normal part.
    """
    r = np.asarray(r, dtype=np.float64)
    v0, v1, v2 = tv[:, 0], tv[:, 1], tv[:, 2]
    n = np.cross(v1 - v0, v2 - v0)
    n = n / np.sqrt(_dot(n, n))[:, None]
    d = _dot(r - v0, n)
    rho = r - d[:, None] * n
    ad = np.abs(d)
    out = np.zeros((len(r), 3))
    bsum = np.zeros(len(r))
    verts = (v0, v1, v2)
    for e in range(3):
        pa, pb = verts[e], verts[(e + 1) % 3]
        L = pb - pa
        s = L / np.sqrt(_dot(L, L))[:, None]
        u = np.cross(s, n)
        lp = _dot(pb - rho, s)
        lm = _dot(pa - rho, s)
        t0 = _dot(pa - rho, u)
        R0sq = t0 * t0 + d * d
        Rp = np.sqrt(lp * lp + R0sq)
        Rm = np.sqrt(lm * lm + R0sq)
        with np.errstate(divide="ignore", invalid="ignore"):
            F = np.where(lp + lm >= 0.0,
                         np.log((Rp + lp) / (Rm + lm)),
                         np.log((Rm - lm) / (Rp - lp)))
            F = np.where(R0sq > 0.0, F, 0.0)
            den_p = R0sq + ad * Rp
            den_m = R0sq + ad * Rm
            beta = np.where(den_p > 0.0, np.arctan(t0 * lp / np.where(den_p > 0, den_p, 1.0)), 0.0) \
                - np.where(den_m > 0.0, np.arctan(t0 * lm / np.where(den_m > 0, den_m, 1.0)), 0.0)
        out += u * F[:, None]
        bsum += beta
    out += n * (np.sign(d) * bsum)[:, None]
    return out
