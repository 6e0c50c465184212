"""Pins for the oracle's EFIE entries and the Mie reference.

The entries are checked against an independent brute-force evaluation of the
defining double integral (refined product quadrature for separated pairs,
polar integration about each observation point for the self pair), against
exact symmetry, and -- through a dense solve -- against the Mie series of a
PEC sphere.  The Mie code is checked against its Rayleigh and optical limits,
energy conservation and the angular integral of its amplitude functions.
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import mie
from oracle.constants import EPS0, MU0, wavenumber
from oracle.efie import EFIEOperator
from oracle.planewave import bistatic_rcs, excitation, monostatic_rcs
from oracle.quadrature import RULE7
from oracle.rwg import build_rwg
from workloads import icosphere

GX, GW = np.polynomial.legendre.leggauss(24)
GX, GW = 0.5 * (GX + 1.0), 0.5 * GW


def _subdivide(tv, lev):
    if lev == 0:
        return [tv]
    a, b, c = tv
    ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
    out = []
    for t in ([a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]):
        out += _subdivide(np.array(t), lev - 1)
    return out


def _area(tv):
    return 0.5 * np.linalg.norm(np.cross(tv[1] - tv[0], tv[2] - tv[0]))


def _brute_pair(k, w, Tm, vm, Tn, vn, lev):
    """int int [ (jw mu/4)(r - vm).(r' - vn) - (j/(w eps)) ] G over Tm x Tn
    with both triangles subdivided 4^lev times (separated pairs only)."""
    pts_m, wts_m, pts_n, wts_n = [], [], [], []
    for st in _subdivide(Tm, lev):
        pts_m.append(RULE7[0] @ st)
        wts_m.append(RULE7[1] * _area(st))
    for st in _subdivide(Tn, lev):
        pts_n.append(RULE7[0] @ st)
        wts_n.append(RULE7[1] * _area(st))
    pm, wm = np.concatenate(pts_m), np.concatenate(wts_m)
    pn, wn = np.concatenate(pts_n), np.concatenate(wts_n)
    R = np.linalg.norm(pm[:, None] - pn[None], axis=2)
    G = np.exp(-1j * k * R) / (4 * math.pi * R)
    dot = (pm - vm) @ (pn - vn).T
    return np.sum(wm[:, None] * wn[None] * G * ((1j * w * MU0 / 4) * dot - 1j / (w * EPS0)))


def _brute_self(k, w, T, vm, lev):
    """Same-triangle term: inner integral in polar coordinates about each
    (in-plane) observation point, outer subdivided 4^lev times."""
    n = np.cross(T[1] - T[0], T[2] - T[0])
    n /= np.linalg.norm(n)
    e1 = (T[1] - T[0]) / np.linalg.norm(T[1] - T[0])
    e2 = np.cross(n, e1)
    tot = 0j
    for st in _subdivide(T, lev):
        ast = _area(st)
        for r, wq in zip(RULE7[0] @ st, RULE7[1]):
            S, V = 0j, np.zeros(3, complex)
            for e in range(3):
                a, b = T[e] - r, T[(e + 1) % 3] - r
                ta = math.atan2(a @ e2, a @ e1)
                dth = math.atan2(b @ e2, b @ e1) - ta
                dth = (dth + math.pi) % (2 * math.pi) - math.pi
                L = b - a
                for u, wu in zip(GX, GW):
                    th = ta + u * dth
                    d = math.cos(th) * e1 + math.sin(th) * e2
                    M = np.array([[d @ e1, -(L @ e1)], [d @ e2, -(L @ e2)]])
                    s_edge = np.linalg.solve(M, np.array([a @ e1, a @ e2]))[0]
                    rr = s_edge * GX
                    G = np.exp(-1j * k * rr) / (4 * math.pi)          # G * r dr
                    wt = wu * dth * s_edge * GW
                    S += np.sum(wt * G)
                    V += np.sum((wt * G)[:, None] * (r + rr[:, None] * d - vm), axis=0)
            tot += ast * wq * ((1j * w * MU0 / 4) * np.dot(r - vm, V) - 1j / (w * EPS0) * S)
    return tot


@pytest.fixture(scope="module")
def sub2():
    xyz, tri = icosphere(2)
    rwg = build_rwg(xyz, tri)
    return rwg, EFIEOperator(rwg, 300e6)


def test_symmetric_exactly(sub2):
    rwg, op = sub2
    Z = op.dense()
    assert np.array_equal(Z, Z.T)
    n = np.arange(3, rwg["N"], 11)
    m = np.arange(0, rwg["N"], 7)[: len(n)]
    assert np.array_equal(op.entries(m, n), op.entries(n, m))


def test_separated_pairs_vs_brute_force(sub2):
    rwg, op = sub2
    xyz, tri = rwg["xyz"], rwg["tri"]
    k, w = op.k, 2 * math.pi * op.freq_hz
    mid = 0.5 * (xyz[rwg["edges"][:, 0]] + xyz[rwg["edges"][:, 1]])
    for m in (0, 200):
        d = np.linalg.norm(mid - mid[m], axis=1)
        for n in np.argsort(d)[[60, 150, 300, 470]]:
            n = int(n)
            ref = 0j
            a, b = min(m, n), max(m, n)
            for sa, tk_a, vk_a in ((1, "tplus", "vplus"), (-1, "tminus", "vminus")):
                for sb, tk_b, vk_b in ((1, "tplus", "vplus"), (-1, "tminus", "vminus")):
                    Ta, Tb = xyz[tri[rwg[tk_a][a]]], xyz[tri[rwg[tk_b][b]]]
                    I = _brute_pair(k, w, Ta, xyz[rwg[vk_a][a]], Tb, xyz[rwg[vk_b][b]], 2)
                    ref += sa * sb * rwg["length"][a] * rwg["length"][b] / (_area(Ta) * _area(Tb)) * I
            val = op.entries(np.array([m]), np.array([n]))[0]
            # accuracy of the 7x7 / 3x3 product rules on these separations
            assert abs(val - ref) <= 5e-3 * abs(ref), (m, n, val, ref)


def test_self_term_vs_polar_brute_force(sub2):
    rwg, op = sub2
    xyz, tri = rwg["xyz"], rwg["tri"]
    k, w = op.k, 2 * math.pi * op.freq_hz
    m = 0
    ours, ref = 0j, 0j
    for sa in (0, 1):
        P = op.t_of[m, sa]
        M0, Ma, Mb, Mab = op.pair_moments(np.array([P]), np.array([P]))
        d = op.cen[P] - op.v_of[m, sa]
        Vv = Mab[0] + d @ Mb[0] + d @ Ma[0] + (d @ d) * M0[0]
        coef = rwg["length"][m] ** 2 / op.area[P] ** 2
        ours += coef * (op.cA * Vv + op.cPhi * M0[0])
        ref += coef * _brute_self(k, w, xyz[tri[P]], op.v_of[m, sa], 1)
    # The 7-point rule on the bounded but non-smooth remainder (exp(-jkR)-1)/R
    # and the 7-point outer rule limit the self term to about 1 percent.
    assert abs(ours.real - ref.real) <= 1e-4 * abs(ref)
    assert abs(ours - ref) <= 1.5e-2 * abs(ref)


def test_mie_limits_and_conservation():
    x = 0.01
    assert abs(mie.backscatter_efficiency(x) / (9 * x ** 4) - 1.0) < 1e-3
    assert abs(mie.backscatter_efficiency(400.0) - 1.0) < 0.02
    for x in (0.3, 2.0, 4.19, 16.6):
        qext, qsca = mie.efficiencies(x)
        assert abs(qext - qsca) < 1e-10 * qsca
        # Q_sca = x^-2 int (|S1|^2 + |S2|^2) sin t dt  (pins pi_n, tau_n)
        f = lambda t: float(np.sum(np.abs(np.array(mie.amplitudes(x, np.array([t])))) ** 2)) * math.sin(t)
        ang = integrate.quad(f, 0, math.pi, limit=400, epsabs=1e-12, epsrel=1e-10)[0] / x ** 2
        assert abs(ang - qsca) < 1e-7 * qsca
        # backscatter from the amplitude function at t = pi
        S1, S2 = mie.amplitudes(x, np.array([math.pi]))
        assert abs(4 * abs(S1[0]) ** 2 / x ** 2 - mie.backscatter_efficiency(x)) < 1e-10 * mie.backscatter_efficiency(x)
        assert abs(abs(S1[0]) - abs(S2[0])) < 1e-12 * abs(S1[0])


def test_dense_efie_sphere_vs_mie(c0_workload, c0_hmatrix, c0_dense):
    """Whole EFIE chain (RWG, quadrature, excitation, RCS) against Mie on the
    1,920-unknown sphere at ka = 4.19: backscatter within 0.5 dB, bistatic
    E-plane RMS within 1 dB away from deep nulls."""
    w = c0_workload
    rwg = c0_hmatrix.rwg
    b = excitation(rwg, w["freq_hz"], w["khat"], w["pol"])
    x = np.linalg.solve(c0_dense, b)
    k = wavenumber(w["freq_hz"])
    s = monostatic_rcs(rwg, w["freq_hz"], w["khat"], w["pol"], x)[0]
    assert abs(10 * np.log10(s / mie.backscatter_rcs(1.0, k))) < 0.5
    th = np.deg2rad(np.arange(0.0, 181.0, 5.0))
    rh = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    ev = np.stack([np.cos(th), 0 * th, -np.sin(th)], 1)
    sb = 10 * np.log10(bistatic_rcs(rwg, w["freq_hz"], x[:, 0], rh, ev))
    sm = 10 * np.log10(mie.bistatic_rcs(1.0, k, math.pi - th, "E"))
    keep = sm > sm.max() - 20
    assert np.sqrt(np.mean((sb - sm)[keep] ** 2)) < 1.0


def test_open_plate_broadside_matches_physical_optics():
    """Open PEC sheet (the square plate of Sec. V.C.2, here 2 wavelengths at
    lambda/10): the dense EFIE solution's broadside backscatter is close to the
    physical-optics value 4 pi A^2 / lambda^2, the large-plate limit (edge
    diffraction of a 2-lambda plate moves it by a few tenths of a dB)."""
    from workloads import workload
    w = workload("plate_2lambda_300MHz")
    rwg = build_rwg(w["xyz"], w["tri"], allow_open=True)
    assert rwg["N"] == 3 * 20 * 20 - 2 * 20          # interior edges of the 20 x 20 grid
    op = EFIEOperator(rwg, w["freq_hz"])
    khat, pol = w["khat"][:1], w["pol"][:1]           # theta = 0: normal incidence
    x = np.linalg.solve(op.dense(), excitation(rwg, w["freq_hz"], khat, pol))
    sig = monostatic_rcs(rwg, w["freq_hz"], khat, pol, x)[0]
    lam = 299792458.0 / w["freq_hz"]
    po = 4.0 * np.pi * (2.0 * lam) ** 4 / lam ** 2
    assert abs(10.0 * np.log10(sig / po)) < 1.0
