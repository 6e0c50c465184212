"""Galerkin EFIE matrix entries with RWG basis and testing (eqs. 2-3, 9).

With the e^{jwt} convention (see ``constants``) the mixed-potential EFIE
tested with f_m gives

  Z_mn = j w mu  int int f_m(r) . f_n(r') G dS' dS
         - (j / (w eps)) int int (div f_m)(div' f_n) G dS' dS,
  G = exp(-j k R) / (4 pi R),

and the excitation b_m = <f_m, E_inc>.  Each entry is a sum over the four
triangle pairs (T_m^+-, T_n^+-).  Writing f = s (l / 2A)(r - v) on a triangle
(s = +-1) gives per pair

  s_m s_n l_m l_n / (A_P A_Q) [ (j w mu / 4) Vv  - (j / (w eps)) S ],
  Vv = int int (r - v_m).(r' - v_n) G,   S = int int G.

Both are formed from four moments of G about the centroids c_P, c_Q of the
outer (test) triangle P and inner (source) triangle Q:
M0 = int int G, Ma = int int (r - c_P) G, Mb = int int (r' - c_Q) G and
Mab = int int (r - c_P).(r' - c_Q) G, so that with dP = c_P - v_m,
dQ = c_Q - v_n:  Vv = Mab + dP.Mb + dQ.Ma + (dP.dQ) M0.

Numerical rules (the paper does not give its quadrature):
* the triangle with the smaller index is the outer one;
* pairs that share a vertex, or whose centroids are closer than 2h (h = the
  longest mesh edge): Radon 7-point outer rule, inner integral = closed form
  of the 1/R part (``potentials``) + 7-point rule on (exp(-jkR) - 1)/R;
* centroid distance < 4h: 7 x 7 points;  otherwise 3 x 3 points.

Only entries with m <= n are evaluated; Z_nm is defined as Z_mn, so Z = Z^T
holds exactly (the symmetry the paper relies on to store only the right
scaling coefficients).  The four triangle-pair terms are summed in the order
(+,+), (+,-), (-,+), (-,-) of (min(m,n), max(m,n)).
"""

import math

import numpy as np

from .constants import MU0, EPS0, wavenumber, omega
from .potentials import triangle_potentials
from .quadrature import RULE3, RULE7, points
from .rwg import triangle_geometry, max_edge_length


def _dot(a, b):
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


class EFIEOperator:
    """Entry evaluator for the EFIE Galerkin matrix of one mesh/frequency."""

    CHUNK = 20000

    def __init__(self, rwg, freq_hz):
        self.rwg = rwg
        self.xyz = rwg["xyz"]
        self.tri = rwg["tri"]
        self.tv = self.xyz[self.tri]
        self.cen, self.area, _ = triangle_geometry(self.xyz, self.tri)
        self.h = max_edge_length(self.xyz, self.tri)
        self.k = wavenumber(freq_hz)
        w = omega(freq_hz)
        self.cA = 1j * w * MU0 / 4.0
        self.cPhi = -1j / (w * EPS0)
        self.freq_hz = freq_hz
        N = rwg["N"]
        # per unknown and side (0: +, 1: -): triangle, free vertex, sign
        self.t_of = np.stack([rwg["tplus"], rwg["tminus"]], axis=1)
        self.v_of = np.stack([self.xyz[rwg["vplus"]], self.xyz[rwg["vminus"]]], axis=1)
        self.s_of = np.array([1.0, -1.0])
        self.N = N

    # ------------------------------------------------------------------ pairs
    def classify(self, O, I):
        """Rule per canonical pair: 0 = singular extraction, 1 = 7x7, 2 = 3x3."""
        to, ti = self.tri[O], self.tri[I]
        share = np.zeros(len(O), dtype=bool)
        for a in range(3):
            for b in range(3):
                share |= to[:, a] == ti[:, b]
        dc = self.cen[O] - self.cen[I]
        d2 = _dot(dc, dc)
        h = self.h
        rule = np.full(len(O), 2, dtype=np.int64)
        rule[d2 < (4.0 * h) * (4.0 * h)] = 1
        rule[share | (d2 < (2.0 * h) * (2.0 * h))] = 0
        return rule

    def _regular(self, O, I, ro_rule, ri_rule):
        k = self.k
        ro = points(self.tv[O], ro_rule)
        ri = points(self.tv[I], ri_rule)
        a = ro - self.cen[O][:, None, :]
        b = ri - self.cen[I][:, None, :]
        D = ro[:, :, None, :] - ri[:, None, :, :]
        R = np.sqrt(_dot(D, D))
        G = np.exp(-1j * k * R) / (4.0 * math.pi * R)
        W = (ro_rule[1][:, None] * ri_rule[1][None, :])[None] * (self.area[O] * self.area[I])[:, None, None]
        WG = W * G
        M0 = WG.sum(axis=(1, 2))
        Ma = np.einsum("pab,pad->pd", WG, a)
        Mb = np.einsum("pab,pbd->pd", WG, b)
        Mab = np.einsum("pab,pab->p", WG, np.einsum("pad,pbd->pab", a, b))
        return M0, Ma, Mb, Mab

    def _singular(self, O, I):
        k = self.k
        P = len(O)
        wo = RULE7[1]
        wi = RULE7[1]
        ro = points(self.tv[O], RULE7)                    # (P, 7, 3)
        ri = points(self.tv[I], RULE7)
        a = ro - self.cen[O][:, None, :]
        b = ri - self.cen[I][:, None, :]
        tvI = np.repeat(self.tv[I], 7, axis=0)
        I1, Irho, rho = triangle_potentials(ro.reshape(-1, 3), tvI)
        I1 = I1.reshape(P, 7)
        cI = np.repeat(self.cen[I], 7, axis=0)
        J = (Irho + (rho - cI) * I1.reshape(-1)[:, None]).reshape(P, 7, 3)
        D = ro[:, :, None, :] - ri[:, None, :, :]
        R = np.sqrt(_dot(D, D))
        # (exp(-jkR) - 1) / (4 pi R) = (-jk / 4pi) * sinc(kR/2) * exp(-jkR/2)
        g = (-1j * k / (4.0 * math.pi)) * np.sinc(k * R / (2.0 * math.pi)) * np.exp(-0.5j * k * R)
        AI = self.area[I][:, None]
        inner_s = I1 / (4.0 * math.pi) + AI * np.einsum("pab,b->pa", g, wi)
        inner_v = J / (4.0 * math.pi) + AI[:, :, None] * np.einsum("pab,b,pbd->pad", g, wi, b)
        AO = self.area[O]
        M0 = AO * np.einsum("a,pa->p", wo, inner_s)
        Ma = AO[:, None] * np.einsum("a,pa,pad->pd", wo, inner_s, a)
        Mb = AO[:, None] * np.einsum("a,pad->pd", wo, inner_v)
        Mab = AO * np.einsum("a,pad,pad->p", wo, a, inner_v)
        return M0, Ma, Mb, Mab

    def pair_moments(self, O, I):
        """Moments (M0, Ma, Mb, Mab) for canonical pairs O <= I (outer O)."""
        O = np.asarray(O, dtype=np.int64)
        I = np.asarray(I, dtype=np.int64)
        P = len(O)
        M0 = np.zeros(P, dtype=np.complex128)
        Ma = np.zeros((P, 3), dtype=np.complex128)
        Mb = np.zeros((P, 3), dtype=np.complex128)
        Mab = np.zeros(P, dtype=np.complex128)
        rule = self.classify(O, I)
        for r in (0, 1, 2):
            idx = np.nonzero(rule == r)[0]
            for c0 in range(0, len(idx), self.CHUNK):
                sel = idx[c0:c0 + self.CHUNK]
                if r == 0:
                    out = self._singular(O[sel], I[sel])
                elif r == 1:
                    out = self._regular(O[sel], I[sel], RULE7, RULE7)
                else:
                    out = self._regular(O[sel], I[sel], RULE3, RULE3)
                M0[sel], Ma[sel], Mb[sel], Mab[sel] = out
        return M0, Ma, Mb, Mab

    # ---------------------------------------------------------------- entries
    def entries(self, m, n):
        """Z_mn for arrays of unknown indices (any shape); Z_nm == Z_mn."""
        m = np.asarray(m, dtype=np.int64)
        n = np.asarray(n, dtype=np.int64)
        shape = np.broadcast(m, n).shape
        a = np.minimum(m, n).reshape(-1)
        b = np.maximum(m, n).reshape(-1)
        out = np.zeros(a.size, dtype=np.complex128)
        step = 4 * self.CHUNK
        for c0 in range(0, a.size, step):
            out[c0:c0 + step] = self._entries_canonical(a[c0:c0 + step], b[c0:c0 + step])
        return out.reshape(shape)

    def _entries_canonical(self, a, b):
        nt = len(self.tri)
        terms = []
        for sa in (0, 1):
            for sb in (0, 1):
                P = self.t_of[a, sa]
                Q = self.t_of[b, sb]
                terms.append((sa, sb, P, Q))
        keys = np.concatenate([np.minimum(P, Q) * nt + np.maximum(P, Q) for _, _, P, Q in terms])
        ukeys, inv = np.unique(keys, return_inverse=True)
        M0, Ma, Mb, Mab = self.pair_moments(ukeys // nt, ukeys % nt)
        out = np.zeros(len(a), dtype=np.complex128)
        la, lb = self.rwg["length"][a], self.rwg["length"][b]
        for t, (sa, sb, P, Q) in enumerate(terms):
            u = inv[t * len(a):(t + 1) * len(a)]
            dA = self.cen[P] - self.v_of[a, sa]
            dB = self.cen[Q] - self.v_of[b, sb]
            pq = P <= Q
            dO = np.where(pq[:, None], dA, dB)
            dI = np.where(pq[:, None], dB, dA)
            Vv = Mab[u] + _dot(dO, Mb[u]) + _dot(dI, Ma[u]) + _dot(dO, dI) * M0[u]
            coef = self.s_of[sa] * self.s_of[sb] * la * lb / (self.area[P] * self.area[Q])
            out = out + coef * (self.cA * Vv + self.cPhi * M0[u])
        return out

    def block(self, rows, cols):
        """Dense block Z[rows][:, cols]."""
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        return self.entries(rows[:, None], cols[None, :])

    def dense(self):
        """The full N x N Galerkin matrix (tiny meshes only)."""
        N = self.N
        iu, ju = np.triu_indices(N)
        vals = self.entries(iu, ju)
        Z = np.zeros((N, N), dtype=np.complex128)
        Z[iu, ju] = vals
        Z[ju, iu] = vals
        return Z
