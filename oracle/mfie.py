"""Galerkin MFIE and CFIE matrix entries with RWG basis and testing
(eqs. 4-9).

MFIE (eq. 6) with the e^{jwt} convention of ``constants``: the current J on a
closed surface with outward unit normal n satisfies

  J/2 - n x PV int J(r') x grad' G dS' = n x H_inc,
  grad' G = (jk + 1/R) G R_hat = (1 + jkR) exp(-jkR) / (4 pi R^3) (r - r')

(eq. 7, R_hat = (r - r')/R).  Testing with f_m gives

  Z^M_mn = 1/2 <f_m, f_n> - <f_m, n x int f_n(r') x grad' G dS'>,
  b^M_m  = <f_m, n x H_inc>.

On the source triangle Q, f_n = s (l / 2A_Q)(r' - v) and
(r' - v) x (r - r') = (r - v) x (r - r'), so the inner integral is
s (l / 2A_Q) (r - v) x W_Q(r) with W_Q(r) = int_Q (r - r') g(R) dS',
g = (1 + jkR) exp(-jkR) / (4 pi R^3).  With a = r - v_m, b = r - v_n and the
identity a . (n x (b x W)) = (a.b)(n.W) - (a.W)(n.b), each triangle pair
(P = test, Q = source) contributes

  P == Q:  + 1/2 c int_P (r - v_m).(r - v_n) dS            (7-point rule, exact)
  P != Q:  - c int_P [(a.b)(n_P.W_Q) - (a.W_Q)(n_P.b)] dS,
  c = s_m s_n l_m l_n / (4 A_P A_Q).

On one flat triangle f_n x (r - r') is normal to it, so n x (.) vanishes and
the principal-value integral over P == Q is zero.

Numerical rules (the paper gives none; chosen like the EFIE's, ``efie``):
* pairs that share a vertex, or with centroids closer than 2h: 7-point outer
  rule; W_Q = (1/4pi) int_Q (r - r')/R^3 dS' in closed form
  (``potentials.triangle_gradient_potential``) + 7-point rule on the bounded
  remainder (r - r') [(1 + jkR) exp(-jkR) - 1] / (4 pi R^3);
* centroid distance < 4h: 7 x 7 points on the full kernel; else 3 x 3.

CFIE (eq. 8): Z^C = alpha Z^E + eta0 (1 - alpha) Z^M and
b^C = alpha b^E + eta0 (1 - alpha) b^M; the paper takes alpha = 0.5 for
closed bodies.  The matrix is not symmetric.
"""

import math

import numpy as np

from .constants import ETA0, wavenumber
from .efie import EFIEOperator
from .potentials import triangle_gradient_potential
from .quadrature import RULE3, RULE7, points
from .rwg import triangle_geometry, max_edge_length


def _dot(a, b):
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def triangle_normals(xyz, tri):
    """Unit normals from the vertex order (outward for counter-clockwise
    triangles seen from outside)."""
    tv = xyz[tri]
    n = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
    return n / np.sqrt(_dot(n, n))[:, None]


def _kernel_parts(k, R):
    """g(R) = (1 + jkR) exp(-jkR) / (4 pi R^3) and its part without the
    static 1/(4 pi R^3)."""
    x = k * R
    c, s = np.cos(x), np.sin(x)
    num_dyn = (c - 1.0 + x * s) + 1j * (x * c - s)      # (1 + jx) e^{-jx} - 1
    den = 4.0 * math.pi * R ** 3
    return (1.0 + num_dyn) / den, num_dyn / den


class MFIEOperator:
    """Entry evaluator for the MFIE Galerkin matrix of one closed mesh."""

    CHUNK = 20000

    def __init__(self, rwg, freq_hz):
        self.rwg = rwg
        self.xyz = rwg["xyz"]
        self.tri = rwg["tri"]
        self.tv = self.xyz[self.tri]
        self.cen, self.area, _ = triangle_geometry(self.xyz, self.tri)
        self.nrm = triangle_normals(self.xyz, self.tri)
        self.h = max_edge_length(self.xyz, self.tri)
        self.k = wavenumber(freq_hz)
        self.t_of = np.stack([rwg["tplus"], rwg["tminus"]], axis=1)
        self.v_of = np.stack([self.xyz[rwg["vplus"]], self.xyz[rwg["vminus"]]], axis=1)
        self.s_of = np.array([1.0, -1.0])
        self.N = rwg["N"]

    def classify(self, P, Q):
        """0 = closed-form static part, 1 = 7 x 7, 2 = 3 x 3 (as the EFIE)."""
        tp, tq = self.tri[P], self.tri[Q]
        share = np.zeros(len(P), dtype=bool)
        for a in range(3):
            for b in range(3):
                share |= tp[:, a] == tq[:, b]
        dc = self.cen[P] - self.cen[Q]
        d2 = _dot(dc, dc)
        rule = np.full(len(P), 2, dtype=np.int64)
        rule[d2 < (4.0 * self.h) ** 2] = 1
        rule[share | (d2 < (2.0 * self.h) ** 2)] = 0
        return rule

    def _W(self, P, Q, rule):
        """Outer points (K, 7, 3), weights times A_P (K, 7), W_Q at them."""
        K = len(P)
        orule = RULE3 if rule == 2 else RULE7
        irule = RULE3 if rule == 2 else RULE7
        ro = points(self.tv[P], orule)
        ri = points(self.tv[Q], irule)
        D = ro[:, :, None, :] - ri[:, None, :, :]            # r - r'
        R = np.sqrt(_dot(D, D))
        g, gdyn = _kernel_parts(self.k, R)
        wi = irule[1][None, None, :] * self.area[Q][:, None, None]
        if rule == 0:
            tvQ = np.repeat(self.tv[Q], 7, axis=0)
            stat = triangle_gradient_potential(ro.reshape(-1, 3), tvQ).reshape(K, 7, 3) / (4.0 * math.pi)
            W = stat + np.einsum("kab,kabd->kad", wi * gdyn, D)
        else:
            W = np.einsum("kab,kabd->kad", wi * g, D)
        wo = orule[1][None, :] * self.area[P][:, None]
        if rule == 2:                                        # pad to 7 points
            pad = np.zeros((K, 4))
            ro = np.concatenate([ro, np.zeros((K, 4, 3))], axis=1)
            W = np.concatenate([W, np.zeros((K, 4, 3), dtype=np.complex128)], axis=1)
            wo = np.concatenate([wo, pad], axis=1)
        return ro, wo, W

    def pair_data(self, P, Q):
        """Outer points, weights and W_Q for ordered pairs P != Q."""
        K = len(P)
        ro = np.zeros((K, 7, 3))
        wo = np.zeros((K, 7))
        W = np.zeros((K, 7, 3), dtype=np.complex128)
        rule = self.classify(P, Q)
        for r in (0, 1, 2):
            idx = np.nonzero(rule == r)[0]
            for c0 in range(0, len(idx), self.CHUNK):
                sel = idx[c0:c0 + self.CHUNK]
                ro[sel], wo[sel], W[sel] = self._W(P[sel], Q[sel], r)
        return ro, wo, W

    def entries(self, m, n):
        """Z^M_mn for arrays of unknown indices (any shape)."""
        m = np.asarray(m, dtype=np.int64)
        n = np.asarray(n, dtype=np.int64)
        shape = np.broadcast(m, n).shape
        a = np.broadcast_to(m, shape).reshape(-1)
        b = np.broadcast_to(n, shape).reshape(-1)
        out = np.zeros(a.size, dtype=np.complex128)
        step = 4 * self.CHUNK
        for c0 in range(0, a.size, step):
            out[c0:c0 + step] = self._entries(a[c0:c0 + step], b[c0:c0 + step])
        return out.reshape(shape)

    def _entries(self, a, b):
        nt = len(self.tri)
        la, lb = self.rwg["length"][a], self.rwg["length"][b]
        combos = [(sa, sb, self.t_of[a, sa], self.t_of[b, sb]) for sa in (0, 1) for sb in (0, 1)]
        keys = np.concatenate([P * nt + Q for _, _, P, Q in combos])
        diff = keys // nt != keys % nt
        ukeys, inv = np.unique(keys[diff], return_inverse=True)
        ro, wo, W = self.pair_data(ukeys // nt, ukeys % nt)
        slot = np.full(keys.size, -1, dtype=np.int64)
        slot[np.nonzero(diff)[0]] = inv
        out = np.zeros(len(a), dtype=np.complex128)
        pts7 = RULE7
        for c, (sa, sb, P, Q) in enumerate(combos):
            sl = slot[c * len(a):(c + 1) * len(a)]
            vm, vn = self.v_of[a, sa], self.v_of[b, sb]
            coef = self.s_of[sa] * self.s_of[sb] * la * lb / (4.0 * self.area[P] * self.area[Q])
            val = np.zeros(len(a), dtype=np.complex128)
            same = sl < 0
            if np.any(same):                                 # 1/2 <f_m, f_n> on the common triangle
                idx = np.nonzero(same)[0]
                rq = points(self.tv[P[idx]], pts7)
                am = rq - vm[idx][:, None, :]
                bn = rq - vn[idx][:, None, :]
                val[idx] = 0.5 * self.area[P[idx]] * np.einsum("q,kq->k", pts7[1], _dot(am, bn))
            if np.any(~same):
                idx = np.nonzero(~same)[0]
                u = sl[idx]
                rq, w, Wq = ro[u], wo[u], W[u]
                am = rq - vm[idx][:, None, :]
                bn = rq - vn[idx][:, None, :]
                nP = self.nrm[P[idx]][:, None, :]
                integrand = _dot(am, bn) * _dot(nP, Wq) - _dot(am, Wq) * _dot(nP, bn)
                val[idx] = -np.einsum("kq,kq->k", w, integrand)
            out = out + coef * val
        return out

    def block(self, rows, cols):
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        return self.entries(rows[:, None], cols[None, :])

    def dense(self):
        i, j = np.meshgrid(np.arange(self.N), np.arange(self.N), indexing="ij")
        return self.entries(i, j)


class CFIEOperator:
    """Z^C = alpha Z^E + eta0 (1 - alpha) Z^M (eq. 8)."""

    def __init__(self, rwg, freq_hz, alpha=0.5):
        self.rwg = rwg
        self.alpha = float(alpha)
        self.E = EFIEOperator(rwg, freq_hz)
        self.M = MFIEOperator(rwg, freq_hz)
        self.N = rwg["N"]

    def entries(self, m, n):
        out = self.alpha * self.E.entries(m, n)
        if self.alpha != 1.0:
            out = out + ETA0 * (1.0 - self.alpha) * self.M.entries(m, n)
        return out

    def block(self, rows, cols):
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        return self.entries(rows[:, None], cols[None, :])

    def dense(self):
        i, j = np.meshgrid(np.arange(self.N), np.arange(self.N), indexing="ij")
        return self.entries(i, j)
