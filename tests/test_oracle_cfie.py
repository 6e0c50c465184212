"""Pins for the oracle's MFIE / CFIE entries (eqs. 4-9) and its
non-symmetric H-matrix, scaling and series.

* the closed-form static MFIE kernel integral against adaptive quadrature;
* MFIE entries of separated and edge-adjacent pairs against a brute-force
  product quadrature of the defining double integral (written without the
  (r' - v) x (r - r') = (r - v) x (r - r') reduction the oracle uses);
* the whole MFIE and CFIE chains (entries, excitation, RCS) against the Mie
  series: backscatter and the bistatic E-plane pattern (a flipped MFIE sign
  or normal gives 10 dB of pattern error);
* the interior resonance: the EFIE and MFIE matrices become ill-conditioned
  near the sphere's first TM interior resonance (ka = 2.744), the CFIE stays
  well-conditioned (the property eq. 8 is used for);
* the non-symmetric H-matrix: accuracy against the dense CFIE matrix, exact
  block diagonality of eq. (23) with separate left coefficients (eq. 18), and
  the two-term series against the dense closed form.
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import mie
from oracle.constants import C0, ETA0, wavenumber
from oracle.efie import EFIEOperator
from oracle.hmatrix import build_hmatrix
from oracle.mfie import MFIEOperator, _kernel_parts
from oracle.planewave import bistatic_rcs, excitation_cfie, monostatic_rcs
from oracle.potentials import triangle_gradient_potential
from oracle.quadrature import RULE7
from oracle.rwg import build_rwg
from oracle.scaling import group_graph, min_degree_order, natural_order, schur_scaling
from oracle.series import PowerSeries, dense_two_term
from workloads import ellipsoid_mesh, icosphere


@pytest.fixture(scope="module")
def sphere480():
    xyz, tri = icosphere(2, 1.0)
    return build_rwg(xyz, tri)


def test_gradient_potential_vs_adaptive_quadrature():
    tv = np.array([[[0.0, 0.0, 0.0], [1.0, 0.1, 0.05], [0.2, 0.9, -0.1]]])
    v0, v1, v2 = tv[0]
    e1, e2 = v1 - v0, v2 - v0
    a2 = np.linalg.norm(np.cross(e1, e2))
    for r in ([0.3, 0.3, 0.4], [0.4, 0.2, -0.15], [1.5, 1.0, 0.3], [0.35, 0.3, 0.05]):
        r = np.array(r)
        got = triangle_gradient_potential(r[None], tv)[0]
        ref = []
        for c in range(3):
            def f(t, s, c=c):
                d = r - (v0 + s * e1 + t * e2)
                return d[c] / np.linalg.norm(d) ** 3 * a2
            ref.append(integrate.dblquad(f, 0, 1, 0, lambda s: 1 - s, epsabs=1e-12, epsrel=1e-11)[0])
        assert np.abs(got - np.array(ref)).max() <= 1e-9 * np.abs(ref).max()


def _subdivide(tv, lev):
    if lev == 0:
        return [tv]
    a, b, c = tv
    ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
    out = []
    for t in ([a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]):
        out += _subdivide(np.array(t), lev - 1)
    return out


def _pts(tv, lev):
    pts, wts = [], []
    for st in _subdivide(tv, lev):
        pts.append(RULE7[0] @ st)
        wts.append(RULE7[1] * 0.5 * np.linalg.norm(np.cross(st[1] - st[0], st[2] - st[0])))
    return np.concatenate(pts), np.concatenate(wts)


def _brute_mfie(rwg, k, m, n, lev):
    """-sum over triangle pairs of int int f_m(r) . [n_P x (f_n(r') x grad' G)]
    plus 1/2 <f_m, f_n>, by product quadrature on 4^lev sub-triangles."""
    xyz, tri = rwg["xyz"], rwg["tri"]
    out = 0.0 + 0.0j
    for tm_key, vm_key, sm in (("tplus", "vplus", 1.0), ("tminus", "vminus", -1.0)):
        for tn_key, vn_key, sn in (("tplus", "vplus", 1.0), ("tminus", "vminus", -1.0)):
            P, Q = rwg[tm_key][m], rwg[tn_key][n]
            vm, vn = xyz[rwg[vm_key][m]], xyz[rwg[vn_key][n]]
            TP, TQ = xyz[tri[P]], xyz[tri[Q]]
            AP = 0.5 * np.linalg.norm(np.cross(TP[1] - TP[0], TP[2] - TP[0]))
            AQ = 0.5 * np.linalg.norm(np.cross(TQ[1] - TQ[0], TQ[2] - TQ[0]))
            fm_c = sm * rwg["length"][m] / (2 * AP)
            fn_c = sn * rwg["length"][n] / (2 * AQ)
            pm, wm = _pts(TP, lev)
            fm = fm_c * (pm - vm)
            if P == Q:
                out += 0.5 * np.sum(wm * np.einsum("qd,qd->q", fm, fn_c * (pm - vn)))
                continue
            nP = np.cross(TP[1] - TP[0], TP[2] - TP[0])
            nP /= np.linalg.norm(nP)
            pn, wn = _pts(TQ, lev)
            fn = fn_c * (pn - vn)
            D = pm[:, None, :] - pn[None, :, :]
            R = np.linalg.norm(D, axis=2)
            g, _ = _kernel_parts(k, R)
            cr = np.cross(fn[None, :, :], D) * g[:, :, None]            # f_n x grad' G
            inner = np.einsum("b,abd->ad", wn, cr)
            out -= np.sum(wm * np.einsum("ad,ad->a", fm, np.cross(nP[None, :], inner)))
    return out


def test_mfie_entries_vs_brute_force(sphere480):
    rwg = sphere480
    f = 300e6
    op = MFIEOperator(rwg, f)
    k = wavenumber(f)
    tp, tm = rwg["tplus"], rwg["tminus"]
    m = 0
    # an edge-adjacent pair (a neighbour sharing a triangle's edge but no triangle)
    tris_m = {tp[m], tm[m]}
    tri = rwg["tri"]
    verts_m = set(tri[tp[m]]) | set(tri[tm[m]])
    adj = [n for n in range(rwg["N"]) if not ({tp[n], tm[n]} & tris_m)
           and len(set(tri[tp[n]]) & verts_m) >= 2]
    # a separated pair (centroid distance well above 4h)
    cen = op.cen
    far = [n for n in range(rwg["N"]) if np.linalg.norm(cen[tp[n]] - cen[tp[m]]) > 6 * op.h][:1]
    share = [n for n in range(rwg["N"]) if n != m and ({tp[n], tm[n]} & tris_m)][:1]
    # separated pair: 3 x 3 rule; pairs through a common triangle and the self
    # entry: closed-form static part + 7 points; edge-adjacent triangles: the
    # static part has a log singularity on the shared edge that the 7-point
    # outer rule resolves to about 6% (the refined reference converges to it)
    for n, lev, tol in ((far[0], 2, 1e-3), (adj[0], 4, 7e-2), (share[0], 4, 5e-3), (m, 4, 5e-3)):
        got = op.entries(np.array([m]), np.array([n]))[0]
        ref = _brute_mfie(rwg, k, m, n, lev)
        assert abs(got - ref) <= tol * abs(ref), (n, got, ref)


def _pattern_error(rwg, f, x):
    k = wavenumber(f)
    th = np.deg2rad(np.arange(0.0, 181.0, 5.0))
    rh = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    ev = np.stack([np.cos(th), 0 * th, -np.sin(th)], 1)
    sb = 10 * np.log10(bistatic_rcs(rwg, f, x, rh, ev))
    sm = 10 * np.log10(mie.bistatic_rcs(1.0, k, math.pi - th, "E"))
    keep = sm > sm.max() - 20
    return np.sqrt(np.mean((sb - sm)[keep] ** 2))


def test_mfie_and_cfie_sphere_vs_mie(sphere480):
    """480-unknown sphere at ka = 4.19 (about lambda/8 edges): backscatter and
    the bistatic E-plane pattern against Mie for the CFIE (alpha = 0.5) and
    the MFIE alone (alpha = 0, the coarser of the two on RWG functions)."""
    rwg = sphere480
    f = 200e6
    khat, pol = np.array([[0.0, 0.0, -1.0]]), np.array([[1.0, 0.0, 0.0]])
    ZE = EFIEOperator(rwg, f).dense()
    ZM = MFIEOperator(rwg, f).dense()
    k = wavenumber(f)
    for alpha, bs_tol, pat_tol in ((0.5, 0.5, 1.0), (0.0, 1.5, 1.2)):
        Z = alpha * ZE + (1 - alpha) * ETA0 * ZM
        x = np.linalg.solve(Z, excitation_cfie(rwg, f, khat, pol, alpha))
        s = monostatic_rcs(rwg, f, khat, pol, x)[0]
        assert abs(10 * np.log10(s / mie.backscatter_rcs(1.0, k))) < bs_tol
        assert _pattern_error(rwg, f, x[:, 0]) < pat_tol


def test_cfie_removes_interior_resonance(sphere480):
    rwg = sphere480
    conds = {0.0: [], 0.5: [], 1.0: []}
    for ka in 2.7437 * np.array([0.97, 0.985, 1.0, 1.015, 1.03]):
        f = ka * C0 / (2 * math.pi)
        ZE = EFIEOperator(rwg, f).dense()
        ZM = MFIEOperator(rwg, f).dense()
        for alpha in conds:
            sv = np.linalg.svd(alpha * ZE + (1 - alpha) * ETA0 * ZM, compute_uv=False)
            conds[alpha].append(sv[0] / sv[-1])
    assert max(conds[1.0]) > 100 and max(conds[0.0]) > 100
    assert max(conds[0.5]) < 5


@pytest.fixture(scope="module")
def cfie_h():
    xyz, tri = icosphere(2, 1.0)
    xyz, tri = ellipsoid_mesh(xyz, tri, (1.3, 0.9, 0.6))
    return build_hmatrix(xyz, tri, 300e6, 16, 1e-3, workers=8, formulation="cfie", alpha=0.5)


def test_cfie_hmatrix_scaling_and_series(cfie_h):
    H = cfie_h
    assert not H.symmetric
    P = H.perm
    Z = H.op.dense()[np.ix_(P, P)]
    ZN, ZF = H.dense_near(), H.dense_far()
    assert np.linalg.norm(ZN + ZF - Z) <= 5e-4 * np.linalg.norm(Z)
    assert np.linalg.norm(ZN - ZN.T) > 1e-2 * np.linalg.norm(ZN)          # genuinely non-symmetric
    b = H.to_tree(excitation_cfie(H.rwg, 300e6, np.array([[0, 0, -1.0], [1.0, 0, 0]]),
                                  np.array([[1.0, 0, 0], [0, 1.0, 0]]), 0.5))
    for order in (natural_order(H.M), min_degree_order(group_graph(H))):
        S = schur_scaling(H, order)
        N = H.N
        A, Ap = np.eye(N, dtype=complex), np.eye(N, dtype=complex)
        for i in order:
            ai, api = np.eye(N, dtype=complex), np.eye(N, dtype=complex)
            si = H.group_slice(i)
            for j in S.later[i]:
                sj = H.group_slice(j)
                ai[si, sj] = -S.C[(i, j)]
                api[sj, si] = -S.left(i, j)
            A, Ap = A @ ai, api @ Ap
        T = Ap @ ZN @ A                                                   # eq. (22)
        mask = np.zeros((N, N), dtype=bool)
        for g in range(H.M):
            s = H.group_slice(g)
            mask[s, s] = True
        assert np.abs(T[~mask]).max() <= 1e-12 * np.abs(T).max()         # eq. (23)
        x, _ = PowerSeries(H, S).solve(b, 2)
        xd = dense_two_term(ZN, ZF, b, 2)
        assert np.abs(x - xd).max() <= 1e-11 * np.abs(xd).max()
