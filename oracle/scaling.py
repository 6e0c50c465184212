"""Right scaling coefficients and Schur-complement scaling of the near field
(Sec. III.A, eqs. 14-23).

Groups (octree leaves) are eliminated one at a time in a chosen order.  For
pivot group i with current (already Schur-updated) near-field blocks Z~:

* eq. (16): the right scaling coefficient alpha_i has blocks
  alpha_ij = -Z~_ii^{-1} Z~_ij for every later group j coupled to i
  (N+(i)); this module stores C_ij = Z~_ii^{-1} Z~_ij, so alpha_ij = -C_ij;
* eq. (18): the left coefficient alpha'_i has blocks -Z~_ji Z~_ii^{-1};
  because Z_N = Z_N^T these are the transposes of the right ones (the
  paper's reason to store only the right coefficients, end of Sec. III.A).
  For a non-symmetric near field (the CFIE of eq. 8) they are kept as
  L_ij = Z~_ji Z~_ii^{-1}, alpha'_ji = -L_ij;
* eqs. (19)-(21): alpha'_i Z~ alpha_i zeroes row and column i and replaces
  every pair j, k in N+(i) by Z~_jk - Z~_ji Z~_ii^{-1} Z~_ik.  Pairs that were
  not coupled before become fill-in blocks (kept: "considering fill-in blocks
  for complete ... scaling", and Sloan ordering is used "to reduce the
  fill-in");
* eq. (23): after every group has been a pivot the scaled near field is block
  diagonal with blocks D_i = Z~_ii taken at their elimination.

Reading (the paper is silent): the inverse of Z~_ii is LAPACK's LU with
partial pivoting inside the block (numpy.linalg.inv -> zgesv); no pivoting
across blocks.  Breakdown: a block is numerically singular when a pivot of
that LU (a diagonal entry of U) has modulus below n eps max|Z~_ii| (n the
block size, eps = 2^-52); the elimination stops there with an error.  The elimination order is any fill-reducing order; this module
uses minimum degree on the group graph (or the natural order), deliberately
not the order of the GPU library.  The full two-term result does not depend
on the order (Z_N = U^T D U exactly, see ``series``).
"""

import numpy as np
import scipy.linalg


class SingularBlock(ArithmeticError):
    pass


def pivots_ok(Z):
    """True when every pivot of LU with partial pivoting of the square block Z
    has modulus at least n eps max|Z| (eps = 2^-52)."""
    n = Z.shape[0]
    lu, _ = scipy.linalg.lu_factor(Z, check_finite=False)
    return bool(np.min(np.abs(np.diag(lu))) >= n * 2.0 ** -52 * np.max(np.abs(Z)))


def group_graph(H):
    adj = {g: set() for g in range(H.M)}
    for (t, s) in H.near:
        if t != s:
            adj[t].add(s)
            adj[s].add(t)
    return adj


def natural_order(M):
    return list(range(M))


def min_degree_order(adj):
    """Elimination game on the group graph: repeatedly eliminate the group of
    smallest current degree (lowest index on ties), joining its remaining
    neighbours pairwise."""
    g = {v: set(n) for v, n in adj.items()}
    order = []
    alive = set(g)
    while alive:
        v = min(alive, key=lambda u: (len(g[u]), u))
        nb = g[v]
        for a in nb:
            g[a] |= nb
            g[a].discard(a)
            g[a].discard(v)
        alive.discard(v)
        order.append(v)
        del g[v]
    return order


class Scaling:
    """Result of the Schur scaling: order, D_i = Z~_ii, D_i^{-1}, C_ij (and
    L_ij for a non-symmetric near field)."""

    def __init__(self, order, D, Dinv, C, later, L=None):
        self.order = order
        self.D = D            # g -> scaled diagonal block (eq. 23)
        self.Dinv = Dinv      # g -> its inverse
        self.C = C            # (i, j) -> Z~_ii^{-1} Z~_ij, alpha_ij = -C_ij
        self.later = later    # i -> N+(i) in elimination order
        self.L = L            # (i, j) -> Z~_ji Z~_ii^{-1} (None: C_ij^T)

    def left(self, i, j):
        """L_ij = Z~_ji Z~_ii^{-1}, so that alpha'_ji = -L_ij (eq. 18)."""
        return self.C[(i, j)].T if self.L is None else self.L[(i, j)]

    def coefficient_entries(self):
        return sum(B.size for B in self.C.values())


def schur_scaling(H, order, rcond_min=0.0):
    """Scale the near field of ``H`` to block-diagonal form (eqs. 16-23).

    The working matrix keeps both triangles (Z~_ij and Z~_ji) so that eq. (21)
    is applied literally, Z~_jk -= Z~_ji (Z~_ii^{-1} Z~_ik), for all j, k in
    N+(i)."""
    symmetric = getattr(H, "symmetric", True)
    W = {}
    for (t, s), B in H.near.items():
        W[(t, s)] = B.copy()
        if t != s and symmetric:
            W[(s, t)] = B.T.copy()
    nbr = group_graph(H)
    pos = {g: p for p, g in enumerate(order)}
    done = set()
    D, Dinv, C, later = {}, {}, {}, {}
    L = None if symmetric else {}
    for i in order:
        Zii = W[(i, i)]
        if not np.any(Zii) or not pivots_ok(Zii):
            raise SingularBlock("group %d" % i)
        try:
            inv = np.linalg.inv(Zii)
        except np.linalg.LinAlgError as e:
            raise SingularBlock("group %d" % i) from e
        if rcond_min > 0.0 and 1.0 / (np.linalg.norm(Zii, 1) * np.linalg.norm(inv, 1)) < rcond_min:
            raise SingularBlock("group %d" % i)
        Ni = sorted((j for j in nbr[i] if j not in done), key=lambda j: pos[j])
        D[i], Dinv[i], later[i] = Zii, inv, Ni
        for j in Ni:                                   # eq. (16)
            C[(i, j)] = inv @ W[(i, j)]
            if L is not None:                          # eq. (18)
                L[(i, j)] = W[(j, i)] @ inv
        for j in Ni:                                   # eq. (21), incl. fill-in
            Zji = W[(j, i)]
            for k in Ni:
                upd = Zji @ C[(i, k)]
                if (j, k) in W:
                    W[(j, k)] = W[(j, k)] - upd
                else:
                    W[(j, k)] = -upd
        for j in Ni:
            nbr[j].update(k for k in Ni if k != j)
        done.add(i)
        for j in Ni:                                   # row/column i are now zero
            del W[(i, j)], W[(j, i)]
        del W[(i, i)]
    return Scaling(list(order), D, Dinv, C, later, L)
