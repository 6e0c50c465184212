"""Power-series solution (Sec. III.A eqs. 24-36, Sec. III.B eqs. 44-45).

With A = alpha_1 alpha_2 ... alpha_M (right coefficients in elimination
order) the scaled system is A^T (Z_N + Z_F) A x~ = b~ (eqs. 24, 27-29):

* eq. (25): b~ = alpha_M^T ... alpha_1^T b -- alpha_1^T is applied first; for
  pivot i it changes only the later groups: b_j <- b_j - C_ij^T b_i.  For a
  non-symmetric near field the left coefficients of eq. (24) are used,
  b_j <- b_j - L_ij b_i (alpha'_ji = -L_ij, eq. 18);
* eq. (32): b_o = Z~_N^{-1} b~ (block-diagonal D^{-1});
* eq. (31): U v = Z~_N^{-1} A^T Z_F A v;
* eqs. (35)-(36): x~ = b_o - U b_o + U^2 b_o - ..., truncated after ``terms``
  terms (two in the paper);
* eq. (26): x = alpha_1 ... alpha_M x~ -- alpha_M is applied first; for pivot
  i it changes only block i: x_i <- x_i - sum_{j in N+(i)} C_ij x_j;
* eq. (45): the per-RHS ratio ||it_n|| / ||it_{n-1}||, it_n = U^n b_o; the
  paper asks for it to be below 0.1.

Everything is in the H-matrix tree order; ``solve_rwg`` converts to and from
the RWG order of the unknowns.
"""

import numpy as np


class PowerSeries:
    def __init__(self, H, S):
        self.H = H
        self.S = S

    def _sl(self, g):
        return self.H.group_slice(g)

    def alpha_T(self, b):
        """eq. (25): alpha_M^T ... alpha_1^T b."""
        v = np.array(b, dtype=np.complex128, copy=True)
        for i in self.S.order:
            vi = v[self._sl(i)]
            for j in self.S.later[i]:
                v[self._sl(j)] -= self.S.left(i, j) @ vi
        return v

    def alpha(self, xt):
        """eq. (26): alpha_1 ... alpha_M x~."""
        v = np.array(xt, dtype=np.complex128, copy=True)
        for i in reversed(self.S.order):
            acc = v[self._sl(i)]
            for j in self.S.later[i]:
                acc = acc - self.S.C[(i, j)] @ v[self._sl(j)]
            v[self._sl(i)] = acc
        return v

    def Dinv(self, v):
        """Z~_N^{-1} v (eqs. 23, 32)."""
        out = np.empty_like(v, dtype=np.complex128)
        for g in range(self.H.M):
            out[self._sl(g)] = self.S.Dinv[g] @ v[self._sl(g)]
        return out

    def U(self, v):
        """eq. (31)."""
        return self.Dinv(self.alpha_T(self.H.far_matvec(self.alpha(v))))

    def solve(self, b, terms=2):
        """x (tree order) and the ratios ||it_n|| / ||it_{n-1}|| (terms-1, R)."""
        b = np.asarray(b, dtype=np.complex128)
        it = self.Dinv(self.alpha_T(b))                 # it_0 = b_o
        xt = it.copy()
        ratios = []
        for n in range(1, terms):
            nxt = self.U(it)
            ratios.append(np.linalg.norm(nxt, axis=0) / np.linalg.norm(it, axis=0))
            it = nxt
            xt = xt + ((-1) ** n) * it
        return self.alpha(xt), np.array(ratios)

    def solve_rwg(self, b_rwg, terms=2):
        x, ratios = self.solve(self.H.to_tree(b_rwg), terms)
        return self.H.to_rwg(x), ratios


def dense_two_term(ZN, ZF, b, terms=2):
    """Closed form sum_{k<terms} (-Z_N^{-1} Z_F)^k Z_N^{-1} b by dense LU."""
    y = np.linalg.solve(ZN, b)
    x = y.copy()
    t = y
    for n in range(1, terms):
        t = np.linalg.solve(ZN, ZF @ t)
        x = x + ((-1) ** n) * t
    return x
