"""Pins for the oracle's geometry layer: quadrature rules, closed-form
potentials, RWG functions and plane-wave excitation."""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle.potentials import triangle_potentials
from oracle.quadrature import RULE3, RULE7
from oracle.rwg import MeshError, build_rwg, rwg_value, triangle_geometry
from oracle.planewave import excitation, monostatic_rcs, far_field_projection, rcs_from_projection
from workloads import icosphere, flat_plate


def _monomial_exact(a, b):
    # int over {x, y >= 0, x + y <= 1} of x^a y^b = a! b! / (a + b + 2)!
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("rule,deg", [(RULE7, 5), (RULE3, 2)])
def test_quadrature_degree(rule, deg):
    bary, w = rule
    assert abs(w.sum() - 1.0) < 1e-15
    x, y = bary[:, 1], bary[:, 2]
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            q = 0.5 * np.sum(w * x ** a * y ** b)
            assert abs(q - _monomial_exact(a, b)) < 1e-15, (a, b)
    # and not exact one degree higher
    errs = [abs(0.5 * np.sum(w * x ** a * y ** (deg + 1 - a)) - _monomial_exact(a, deg + 1 - a))
            for a in range(deg + 2)]
    assert max(errs) > 1e-6


TRI = np.array([[0.1, 0.2, 0.0], [1.3, 0.1, 0.05], [0.4, 1.1, -0.1]])


def _polar_in_plane(rho, f):
    """int over TRI of f(r') / |r' - rho| for rho in the plane, by splitting
    at rho into three sub-triangles and integrating in polar coordinates
    (the 1/R factor cancels the Jacobian)."""
    tot = 0.0
    for e in range(3):
        pa, pb = TRI[e], TRI[(e + 1) % 3]
        a, b = pa - rho, pb - rho

        def inner(t):
            q = a + t * (b - a)                 # point on the edge
            dq = b - a
            # polar: d(area) = |q x dq| dt * s ds, r' = rho + s q, R = s |q|
            jac = np.linalg.norm(np.cross(q, dq))
            val = integrate.quad(lambda s: f(rho + s * q) / np.linalg.norm(q), 0.0, 1.0,
                                 epsabs=1e-14, epsrel=1e-12)[0]
            return jac * val
        sgn = np.sign(np.dot(np.cross(a, b), np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0])))
        tot += sgn * integrate.quad(inner, 0.0, 1.0, epsabs=1e-14, epsrel=1e-12)[0]
    return tot


def _dblquad(r, f):
    v0, v1, v2 = TRI
    J = np.linalg.norm(np.cross(v1 - v0, v2 - v0))
    return integrate.dblquad(lambda v, u: f(v0 + u * (v1 - v0) + v * (v2 - v0), r) * J,
                             0, 1, 0, lambda u: 1 - u, epsabs=1e-13, epsrel=1e-11)[0]


@pytest.mark.parametrize("r", [[0.5, 0.5, 0.7], [2.0, -1.0, 0.3], [0.6, 0.6, 1e-3]])
def test_potentials_off_plane(r):
    r = np.array(r)
    I1, Ir, rho = triangle_potentials(r[None], TRI[None])
    ref = _dblquad(r, lambda p, r: 1.0 / np.linalg.norm(p - r))
    assert abs(I1[0] - ref) < 1e-9 * abs(ref)
    for c in range(3):
        refc = _dblquad(r, lambda p, r, c=c: (p - rho[0])[c] / np.linalg.norm(p - r))
        assert abs(Ir[0, c] - refc) < 1e-8 * max(1e-3, abs(refc))


def test_potentials_singular_in_plane():
    """Observation points inside and outside the triangle, in its plane."""
    n = np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0])
    n /= np.linalg.norm(n)
    for bary in ([1 / 3, 1 / 3, 1 / 3], [0.7, 0.2, 0.1], [1.4, -0.2, -0.2]):
        rho = np.array(bary) @ TRI
        I1, Ir, prj = triangle_potentials(rho[None], TRI[None])
        assert np.allclose(prj[0], rho, atol=1e-14)
        ref = _polar_in_plane(rho, lambda p: 1.0)
        assert abs(I1[0] - ref) < 1e-9 * abs(ref)
        for c in range(3):
            refc = _polar_in_plane(rho, lambda p, c=c: (p - rho)[c])
            assert abs(Ir[0, c] - refc) < 1e-9 * max(1e-2, abs(refc))


def test_rwg_counts_and_order():
    for s in (1, 2, 3):
        xyz, tri = icosphere(s)
        rwg = build_rwg(xyz, tri)
        assert rwg["N"] == 3 * len(tri) // 2
        assert len(xyz) - rwg["N"] + len(tri) == 2
        ev = rwg["edges"]
        assert np.all(ev[:, 0] < ev[:, 1])
        keys = ev[:, 0] * len(xyz) + ev[:, 1]
        assert np.all(np.diff(keys) > 0)


def test_rwg_flux_continuity():
    """Normal component of f across its edge is +1 from both sides."""
    xyz, tri = icosphere(2)
    rwg = build_rwg(xyz, tri)
    for n in range(0, rwg["N"], 37):
        a, b = xyz[rwg["edges"][n]]
        pts = np.array([a + t * (b - a) for t in (0.1, 0.5, 0.9)])
        vp, vm = xyz[rwg["vplus"][n]], xyz[rwg["vminus"][n]]
        for side, v in ((1, vp), (-1, vm)):
            f = rwg_value(rwg, n, side, pts)
            e = (b - a) / np.linalg.norm(b - a)
            away = (a - v) - np.dot(a - v, e) * e          # normal to the edge, away from v
            away /= np.linalg.norm(away)
            flux = f @ away * side                          # into T- is +side for T+
            assert np.allclose(flux, 1.0, atol=1e-12)
        # T+ traverses the edge from the smaller to the larger vertex id
        t = tri[rwg["tplus"][n]]
        i0 = int(np.nonzero(t == rwg["edges"][n, 0])[0][0])
        assert t[(i0 + 1) % 3] == rwg["edges"][n, 1]


def test_mesh_errors():
    xyz, tri = icosphere(1)
    with pytest.raises(MeshError):
        build_rwg(xyz, tri[1:])                           # open
    bad = tri.copy()
    bad[0] = bad[0][[0, 2, 1]]
    with pytest.raises(MeshError):
        build_rwg(xyz, bad)                               # flipped
    deg = tri.copy()
    deg[0, 1] = deg[0, 0]
    with pytest.raises(MeshError):
        build_rwg(xyz, deg)
    pxyz, ptri = flat_plate(1.0, 4)
    rwg = build_rwg(pxyz, ptri, allow_open=True)
    assert rwg["N"] == (3 * len(ptri) - 4 * 4) // 2   # interior edges only


def test_excitation_static_limit():
    """As k -> 0, b_m -> pol . int f_m dS = pol . (l/3)(v- - v+)."""
    xyz, tri = icosphere(2)
    rwg = build_rwg(xyz, tri)
    pol = np.array([[0.3, -0.5, 0.8]])
    b = excitation(rwg, 1e-6, [[0.0, 0.0, -1.0]], pol)[:, 0]
    ref = (rwg["length"] / 3.0)[:, None] * (xyz[rwg["vminus"]] - xyz[rwg["vplus"]]) @ pol[0]
    assert np.max(np.abs(b - ref)) < 1e-12 * np.max(np.abs(ref))


def test_excitation_vs_refined_quadrature():
    """7-point excitation against a subdivided (4^3 pieces) 7-point rule."""
    xyz, tri = icosphere(1)
    rwg = build_rwg(xyz, tri)
    f = 300e6
    k = 2 * math.pi * f / 299792458.0
    khat = np.array([0.0, 0.6, -0.8])
    pol = np.array([1.0, 0.0, 0.0])
    b = excitation(rwg, f, khat[None], pol[None])[:, 0]
    bary, w = RULE7

    def sub(tv, lev):
        if lev == 0:
            return [tv]
        a, bb, c = tv
        ab, bc, ca = (a + bb) / 2, (bb + c) / 2, (c + a) / 2
        out = []
        for t in ([a, ab, ca], [ab, bb, bc], [ca, bc, c], [ab, bc, ca]):
            out += sub(np.array(t), lev - 1)
        return out
    cen, area, _ = triangle_geometry(xyz, tri)
    for n in range(0, rwg["N"], 11):
        tot = 0.0
        for side, tk, vk in ((1, "tplus", "vplus"), (-1, "tminus", "vminus")):
            T = tri[rwg[tk][n]]
            v = xyz[rwg[vk][n]]
            A = area[rwg[tk][n]]
            for st in sub(xyz[T], 3):
                a_st = 0.5 * np.linalg.norm(np.cross(st[1] - st[0], st[2] - st[0]))
                p = bary @ st
                fv = side * rwg["length"][n] / (2 * A) * (p - v)
                tot += a_st * np.sum(w * (fv @ pol) * np.exp(-1j * k * p @ khat))
        assert abs(b[n] - tot) < 2e-4 * np.max(np.abs(b))


def test_monostatic_rcs_equals_b_dot_x():
    """For a monostatic co-polar look the receive vector is the excitation."""
    xyz, tri = icosphere(2)
    rwg = build_rwg(xyz, tri)
    f = 250e6
    th = np.deg2rad([0.0, 37.0, 90.0])
    khat = -np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    pol = np.stack([np.cos(th), 0 * th, -np.sin(th)], 1)
    b = excitation(rwg, f, khat, pol)
    F = far_field_projection(rwg, f, -khat, pol)
    assert np.max(np.abs(F - b)) < 1e-15 * np.max(np.abs(b)) * 10
    x = np.random.default_rng(1).standard_normal(b.shape) + 0j
    assert np.allclose(monostatic_rcs(rwg, f, khat, pol, x), rcs_from_projection(f, b, x), rtol=1e-14)
