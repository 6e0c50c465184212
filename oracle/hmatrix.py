"""The H-matrix split Z = Z_N + Z_F of eq. (13).

Everything is indexed in *tree order* (position p holds RWG unknown perm[p]):

* groups (leaves) g = 0..M-1 own the contiguous ranges [lo_g, hi_g);
* near blocks (t, s), t <= s, touching leaves, hold the dense Galerkin block
  Z[perm[t], perm[s]]; the (s, t) block is its transpose (Z = Z^T);
* far blocks (t, s), admissible cluster pairs with t before s in depth-first
  order, hold ACA factors with Z[perm[t], perm[s]] ~= U V^T; the (s, t)
  block is V U^T.

The CFIE matrix (eq. 8) is not symmetric: then ``symmetric`` is False, near
blocks are stored for every ordered pair (t, s) of touching leaves and far
blocks for both orders of every admissible pair, each applied only as
Z[t, s] ~= U V^T.
"""

import numpy as np

from .aca import aca
from .cluster import build_tree, block_partition
from .efie import EFIEOperator
from .mfie import CFIEOperator
from .rwg import build_rwg, edge_midpoints


class HMatrix:
    def __init__(self, N, perm, groups, near, far, symmetric=True):
        self.N = N
        self.perm = np.asarray(perm, dtype=np.int64)
        self.groups = np.asarray(groups, dtype=np.int64)        # (M, 2) lo, hi
        self.near = near    # dict (t, s) -> block, t <= s (all ordered pairs if not symmetric)
        self.far = far      # list of (tlo, thi, slo, shi, U, V)
        self.symmetric = symmetric

    @property
    def M(self):
        return len(self.groups)

    def group_slice(self, g):
        lo, hi = self.groups[g]
        return slice(int(lo), int(hi))

    # ------------------------------------------------------------- products
    def near_matvec(self, x):
        """Z_N x in tree order; x is (N,) or (N, R)."""
        y = np.zeros_like(x, dtype=np.complex128)
        for (t, s), B in self.near.items():
            st, ss = self.group_slice(t), self.group_slice(s)
            y[st] += B @ x[ss]
            if t != s and self.symmetric:
                y[ss] += B.T @ x[st]
        return y

    def far_matvec(self, x):
        """Z_F x in tree order (both directions of every stored block)."""
        y = np.zeros_like(x, dtype=np.complex128)
        for tlo, thi, slo, shi, U, V in self.far:
            y[tlo:thi] += U @ (V.T @ x[slo:shi])
            if self.symmetric:
                y[slo:shi] += V @ (U.T @ x[tlo:thi])
        return y

    def matvec(self, x):
        return self.near_matvec(x) + self.far_matvec(x)

    def dense_near(self):
        Z = np.zeros((self.N, self.N), dtype=np.complex128)
        for (t, s), B in self.near.items():
            st, ss = self.group_slice(t), self.group_slice(s)
            Z[st, ss] = B
            if self.symmetric:
                Z[ss, st] = B.T
        return Z

    def dense_far(self):
        Z = np.zeros((self.N, self.N), dtype=np.complex128)
        for tlo, thi, slo, shi, U, V in self.far:
            B = U @ V.T
            Z[tlo:thi, slo:shi] = B
            if self.symmetric:
                Z[slo:shi, tlo:thi] = B.T
        return Z

    def to_tree(self, x_rwg):
        return np.asarray(x_rwg)[self.perm]

    def to_rwg(self, x_tree):
        out = np.empty_like(x_tree)
        out[self.perm] = x_tree
        return out

    def far_entries(self):
        """sum over both triangles of r (m + n): the applied far entries."""
        f = 2 if self.symmetric else 1
        return sum(f * U.shape[1] * (U.shape[0] + V.shape[0]) for _, _, _, _, U, V in self.far)


_JOB = {}


def _near_job(pairs):
    op, perm = _JOB["op"], _JOB["perm"]
    return [op.block(perm[tlo:thi], perm[slo:shi]) for tlo, thi, slo, shi in pairs]


def _far_job(pairs):
    op, perm, eps = _JOB["op"], _JOB["perm"], _JOB["eps"]
    out = []
    for tlo, thi, slo, shi in pairs:
        rows, cols = perm[tlo:thi], perm[slo:shi]
        out.append(aca(lambda i: op.entries(rows[i], cols),
                       lambda j: op.entries(rows, cols[j]),
                       lambda: op.block(rows, cols),
                       len(rows), len(cols), eps))
    return out


def _init_worker(job):
    _JOB.update(job)
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _run(job, items, workers, chunk=64):
    """Independent blocks over worker processes.  The workers come from a
    fork server (a fresh interpreter), never from a fork of the caller, which
    may hold a GPU runtime with live threads and device mappings; the
    operator and permutation reach them through the pool's initializer."""
    chunks = [items[i:i + chunk] for i in range(0, len(items), chunk)]
    if workers <= 1:
        res = [job(c) for c in chunks]
    else:
        import multiprocessing as mp
        with mp.get_context("forkserver").Pool(workers, initializer=_init_worker, initargs=(dict(_JOB),)) as pool:
            res = pool.map(job, chunks)
    return [r for c in res for r in c]


def build_hmatrix(xyz, tri, freq_hz, leaf_max, aca_tol, eta_far=True, workers=1, box_min=0.0, open_surface=False,
                  formulation="efie", alpha=0.5, eta=2.0):
    """Mesh -> RWG -> octree -> near blocks (quadrature) + far blocks (ACA).

    With ``eta_far=False`` nothing is admissible: every leaf pair becomes a
    near block (Z_F = 0), used to pin the series against a dense LU solve.
    ``eta`` is the admissibility constant of eq. (10) (any value >= sqrt(3):
    far = cells that do not touch).  ``workers`` > 1 evaluates independent blocks in worker processes (the
    arithmetic of each block is unchanged).  ``box_min`` > 0 stops the octree
    at cells of at least that side (metres), whatever their unknown count.
    ``open_surface`` accepts boundary edges (an open PEC sheet such as the
    square plate of Sec. V.C.2), which carry no unknown.  ``formulation``
    "cfie" builds the CFIE matrix of eq. (8) with the given ``alpha`` (closed
    surfaces only); its H-matrix is not symmetric.
    """
    rwg = build_rwg(xyz, tri, allow_open=open_surface)
    if formulation == "efie":
        op = EFIEOperator(rwg, freq_hz)
    elif formulation == "cfie":
        if open_surface:
            raise ValueError("the CFIE needs a closed surface")
        op = CFIEOperator(rwg, freq_hz, alpha)
    else:
        raise ValueError("formulation must be 'efie' or 'cfie'")
    symmetric = formulation == "efie"
    tree = build_tree(edge_midpoints(rwg), leaf_max, box_min)
    perm = tree["perm"]
    leaves = tree["leaves"]
    groups = np.array([(nd.lo, nd.hi) for nd in leaves], dtype=np.int64)
    near_pairs, far_pairs = block_partition(tree, eta)
    if not eta_far:
        near_pairs = [(a, b) for a in leaves for b in leaves if a.leaf_id <= b.leaf_id]
        far_pairs = []
    if not symmetric:
        near_pairs = sorted(near_pairs + [(s, t) for t, s in near_pairs if t.leaf_id != s.leaf_id],
                            key=lambda p: (p[0].leaf_id, p[1].leaf_id))
        far_pairs = sorted(far_pairs + [(s, t) for t, s in far_pairs], key=lambda p: (p[0].id, p[1].id))
    _JOB.update(op=op, perm=perm, eps=aca_tol)
    try:
        nb = _run(_near_job, [(t.lo, t.hi, s.lo, s.hi) for t, s in near_pairs], workers)
        fb = _run(_far_job, [(t.lo, t.hi, s.lo, s.hi) for t, s in far_pairs], workers, chunk=16)
    finally:
        _JOB.clear()
    near = {(t.leaf_id, s.leaf_id): B for (t, s), B in zip(near_pairs, nb)}
    far = [(t.lo, t.hi, s.lo, s.hi, U, V) for (t, s), (U, V) in zip(far_pairs, fb)]
    H = HMatrix(rwg["N"], perm, groups, near, far, symmetric=symmetric)
    H.rwg, H.op, H.tree = rwg, op, tree
    H.near_pairs, H.far_pairs = near_pairs, far_pairs
    return H


def build_hmatrix_cluster(xyz, tri, freq_hz, leaf_max, aca_tol, max_unknowns, workers=1, eta=2.0):
    """The principal sub-H-matrix of one cluster of the full problem (a
    bounded sample of a large workload): the octree and block partition of
    the whole mesh are built as in ``build_hmatrix``; the cluster is the
    largest tree node with at most ``max_unknowns`` unknowns (the first in
    depth-first order among equals).  Its near blocks (both leaves inside the
    cluster) and far blocks (both clusters inside it) are evaluated exactly as
    ``build_hmatrix`` evaluates them, re-indexed from 0.

    Returns (H_sub, info): H_sub in the cluster's local tree order, with
    ``rwg_index`` = the global RWG numbers of its unknowns in that order;
    info = the full problem's leaf sizes, near leaf pairs and far cluster
    pairs (sizes m, n), for scaling the sample's cost to the whole problem."""
    rwg = build_rwg(xyz, tri)
    op = EFIEOperator(rwg, freq_hz)
    tree = build_tree(edge_midpoints(rwg), leaf_max)
    perm, leaves, nodes = tree["perm"], tree["leaves"], tree["nodes"]
    near_pairs, far_pairs = block_partition(tree, eta)
    size = [nd.hi - nd.lo for nd in nodes]
    best = max((nd for nd in nodes if size[nd.id] <= max_unknowns), key=lambda nd: (size[nd.id], -nd.id))
    lo, hi = best.lo, best.hi

    def inside(nd):
        return nd.lo >= lo and nd.hi <= hi

    sub_leaves = [nd for nd in leaves if inside(nd)]
    l0 = sub_leaves[0].leaf_id
    sub_near = [(t, s) for t, s in near_pairs if inside(t) and inside(s)]
    sub_far = [(t, s) for t, s in far_pairs if inside(t) and inside(s)]
    _JOB.update(op=op, perm=perm, eps=aca_tol)
    try:
        nb = _run(_near_job, [(t.lo, t.hi, s.lo, s.hi) for t, s in sub_near], workers)
        fb = _run(_far_job, [(t.lo, t.hi, s.lo, s.hi) for t, s in sub_far], workers, chunk=16)
    finally:
        _JOB.clear()
    groups = np.array([(nd.lo - lo, nd.hi - lo) for nd in sub_leaves], dtype=np.int64)
    near = {(t.leaf_id - l0, s.leaf_id - l0): B for (t, s), B in zip(sub_near, nb)}
    far = [(t.lo - lo, t.hi - lo, s.lo - lo, s.hi - lo, U, V) for (t, s), (U, V) in zip(sub_far, fb)]
    H = HMatrix(hi - lo, np.arange(hi - lo), groups, near, far)
    H.rwg_index = perm[lo:hi].copy()
    info = dict(N=int(rwg["N"]), leaf_sizes=[nd.hi - nd.lo for nd in leaves],
                near_pairs=[(t.leaf_id, s.leaf_id) for t, s in near_pairs],
                far_sizes=[(t.hi - t.lo, s.hi - s.lo) for t, s in far_pairs], rwg=rwg)
    return H, info
