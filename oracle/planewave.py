"""Plane-wave excitation and radar cross-section (Sec. V experiments).

Incident field E_inc(r) = pol * E0 * exp(-j k khat.r) with E0 = 1 V/m.
Excitation (right-hand side of eq. 9): b_m = <f_m, E_inc>, evaluated with the
Radon 7-point rule on T_m^+ and T_m^-.

Far field of a current J = sum_n x_n f_n in direction rhat (e^{jwt}):
  E_far = -j w mu exp(-jkr)/(4 pi r) * [int J exp(+j k rhat.r') dS']_transverse
so sigma = 4 pi r^2 |E_far . e|^2 / |E0|^2 = (k^2 eta^2 / 4 pi) |e . F|^2,
F = sum_n x_n int f_n exp(j k rhat.r') dS'.  For a monostatic look
(rhat = -khat) received in the transmit polarisation (e = pol), e.F equals
b^T x, so sigma_r = (k^2 eta^2 / 4 pi) |b_r^T x_r|^2.
"""

import math

import numpy as np

from .constants import ETA0, wavenumber
from .quadrature import RULE7, points
from .rwg import triangle_geometry


def _rwg_projection(rwg, freq_hz, dirs, vecs, sign):
    """P[n, r] = int f_n . vecs[r] exp(sign * j k dirs[r].r) dS."""
    k = wavenumber(freq_hz)
    xyz, tri = rwg["xyz"], rwg["tri"]
    _, area, _ = triangle_geometry(xyz, tri)
    tv = xyz[tri]
    out = np.zeros((rwg["N"], len(dirs)), dtype=np.complex128)
    for side, tkey, vkey, s in ((0, "tplus", "vplus", 1.0), (1, "tminus", "vminus", -1.0)):
        t = rwg[tkey]
        pts = points(tv[t], RULE7)                             # (N, 7, 3)
        rel = pts - xyz[rwg[vkey]][:, None, :]                 # r - v
        coef = s * rwg["length"] / (2.0 * area[t]) * area[t]   # (l / 2A) * A
        phase = np.exp(sign * 1j * k * np.einsum("nqd,rd->nqr", pts, dirs))
        fdotp = np.einsum("nqd,rd->nqr", rel, vecs)
        out += coef[:, None] * np.einsum("q,nqr->nr", RULE7[1], fdotp * phase)
    return out


def excitation(rwg, freq_hz, khat, pol):
    """b (N, R) for plane waves travelling along khat[r] with polarisation pol[r]."""
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    pol = np.atleast_2d(np.asarray(pol, dtype=np.float64))
    return _rwg_projection(rwg, freq_hz, khat, pol, -1.0)


def far_field_projection(rwg, freq_hz, rhat, evec):
    """F[n, r] = int f_n . evec[r] exp(+j k rhat[r].r) dS (receive vectors)."""
    rhat = np.atleast_2d(np.asarray(rhat, dtype=np.float64))
    evec = np.atleast_2d(np.asarray(evec, dtype=np.float64))
    return _rwg_projection(rwg, freq_hz, rhat, evec, +1.0)


def rcs_from_projection(freq_hz, proj, x):
    """sigma (m^2) for each column: (k^2 eta^2 / 4 pi) |proj[:, r]^T x[:, r]|^2."""
    k = wavenumber(freq_hz)
    amp = np.einsum("nr,nr->r", proj, x)
    return k * k * ETA0 * ETA0 / (4.0 * math.pi) * np.abs(amp) ** 2


def bistatic_rcs(rwg, freq_hz, x, rhat, evec):
    """sigma (m^2) of one current vector x (N,) in the directions rhat (R, 3),
    received along evec (R, 3)."""
    F = far_field_projection(rwg, freq_hz, rhat, evec)
    k = wavenumber(freq_hz)
    amp = F.T @ x
    return k * k * ETA0 * ETA0 / (4.0 * math.pi) * np.abs(amp) ** 2


def monostatic_rcs(rwg, freq_hz, khat, pol, x):
    """sigma (m^2) per RHS for monostatic co-polarised looks."""
    F = far_field_projection(rwg, freq_hz, -np.atleast_2d(khat), pol)
    return rcs_from_projection(freq_hz, F, x)


def dbsm(sigma):
    return 10.0 * np.log10(sigma)


def excitation_cfie(rwg, freq_hz, khat, pol, alpha):
    """CFIE right-hand side (eq. 8): alpha <f_m, E_inc> + eta0 (1 - alpha)
    <f_m, n x H_inc> with eta0 H_inc = khat x E_inc and n the outward normal of
    each triangle; b (N, R)."""
    khat = np.atleast_2d(np.asarray(khat, dtype=np.float64))
    pol = np.atleast_2d(np.asarray(pol, dtype=np.float64))
    k = wavenumber(freq_hz)
    xyz, tri = rwg["xyz"], rwg["tri"]
    _, area, _ = triangle_geometry(xyz, tri)
    tv = xyz[tri]
    nrm = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    hdir = np.cross(khat, pol)                                  # eta0 H_inc / E_inc
    out = np.zeros((rwg["N"], len(khat)), dtype=np.complex128)
    for tkey, vkey, s in (("tplus", "vplus", 1.0), ("tminus", "vminus", -1.0)):
        t = rwg[tkey]
        pts = points(tv[t], RULE7)
        rel = pts - xyz[rwg[vkey]][:, None, :]
        coef = s * rwg["length"] / 2.0                          # (l / 2A) * A
        phase = np.exp(-1j * k * np.einsum("nqd,rd->nqr", pts, khat))
        nxh = np.cross(nrm[t][:, None, :], hdir[None, :, :])    # (N, R, 3)
        vec = alpha * pol[None, :, :] + (1.0 - alpha) * nxh
        fdot = np.einsum("nqd,nrd->nqr", rel, vec)
        out += coef[:, None] * np.einsum("q,nqr->nr", RULE7[1], fdot * phase)
    return out
