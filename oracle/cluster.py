"""Cluster tree and the near/far (admissibility) split.

The paper partitions the geometry with a binary tree and calls a block pair
admissible (far, compressed by ACA) when eta * dist >= min(diam) (eq. 10);
leaf pairs that fail the test form the near field (eq. 13).  The workloads here
fix the leaf size by unknown count, so the tree is an octree:

* points = RWG edge midpoints; root cube [lo, lo + s] with lo the per-axis
  minimum and s = (largest extent) * (1 + 2^-20);
* integer coordinates q = floor((p - lo) / s * 2^21) (clamped to 2^21 - 1);
  a cell at depth d holds the points with q >> (21 - d) equal to its coords;
* a cell is split while it holds more than ``leaf_max`` points (depth <= 21)
  and, when a minimum box side is given, while its children would still be at
  least that wide (electrically sized leaves, Sec. V.A: leaves of at least
  half a wavelength for two-term convergence);
  non-empty children are visited in the order c = 4 bx + 2 by + bz;
* unknowns inside a leaf are ordered by RWG index; the tree order of the
  unknowns is the depth-first order of the leaves.

Admissibility (eq. 10): eta * dist >= min(dia), with cubic cells, dia = the
cell diagonal = sqrt(3) * side and dist = the Euclidean gap between the two
closed cubes, evaluated on the integer coordinates (units of the finest
grid) as 3 s^2 <= eta^2 d^2, s the smaller side, d^2 the squared gap.  With
eta >= sqrt(3) (default 2) this is "the two closed cubes do not touch" (their
gap along some axis is at least the smaller side); eta = 0 admits nothing.
Block-cluster recursion from (root, root): an admissible pair is far; two
inadmissible leaves are near; otherwise the non-leaf (the coarser one, or
both at equal depth) is split.
"""

import numpy as np

DEPTH_MAX = 21


class Node:
    __slots__ = ("depth", "ijk", "pts", "children", "lo", "hi", "id", "leaf_id")

    def __init__(self, depth, ijk, pts):
        self.depth = depth
        self.ijk = ijk
        self.pts = pts
        self.children = []
        self.lo = self.hi = self.id = -1
        self.leaf_id = -1

    @property
    def is_leaf(self):
        return not self.children

    def span(self):
        sh = DEPTH_MAX - self.depth
        return [(c << sh, (c + 1) << sh) for c in self.ijk]


def root_side(points):
    ext = points.max(axis=0) - points.min(axis=0)
    return ext.max() * (1.0 + 2.0 ** -20)


def integer_coords(points):
    lo = points.min(axis=0)
    s = root_side(points)
    q = np.floor((points - lo) / s * float(1 << DEPTH_MAX)).astype(np.int64)
    return np.clip(q, 0, (1 << DEPTH_MAX) - 1)


def depth_limit(side, box_min):
    """Deepest level whose cells are still at least box_min wide."""
    d = 0
    while d < DEPTH_MAX and box_min > 0.0 and side / 2.0 ** (d + 1) >= box_min:
        d += 1
    return d if box_min > 0.0 else DEPTH_MAX


def build_tree(points, leaf_max, box_min=0.0):
    points = np.asarray(points, dtype=np.float64)
    q = integer_coords(points)
    dmax = depth_limit(root_side(points), box_min)
    root = Node(0, (0, 0, 0), np.arange(len(q)))
    stack = [root]
    while stack:
        nd = stack.pop()
        if len(nd.pts) <= leaf_max or nd.depth >= dmax:
            continue
        sh = DEPTH_MAX - nd.depth - 1
        bits = (q[nd.pts] >> sh) & 1
        code = 4 * bits[:, 0] + 2 * bits[:, 1] + bits[:, 2]
        for c in range(8):
            sel = nd.pts[code == c]
            if len(sel) == 0:
                continue
            bx, by, bz = (c >> 2) & 1, (c >> 1) & 1, c & 1
            ijk = (2 * nd.ijk[0] + bx, 2 * nd.ijk[1] + by, 2 * nd.ijk[2] + bz)
            nd.children.append(Node(nd.depth + 1, ijk, sel))
        stack.extend(nd.children)
    # depth-first numbering, tree order of unknowns
    perm, nodes, leaves = [], [], []

    def visit(nd):
        nd.id = len(nodes)
        nodes.append(nd)
        nd.lo = len(perm)
        if nd.is_leaf:
            nd.leaf_id = len(leaves)
            leaves.append(nd)
            perm.extend(sorted(int(p) for p in nd.pts))
        for ch in nd.children:
            visit(ch)
        nd.hi = len(perm)

    import sys
    sys.setrecursionlimit(max(10000, sys.getrecursionlimit()))
    visit(root)
    return dict(root=root, nodes=nodes, leaves=leaves, perm=np.array(perm, dtype=np.int64))


def touch(a, b):
    for (alo, ahi), (blo, bhi) in zip(a.span(), b.span()):
        if alo > bhi or blo > ahi:
            return False
    return True


def admissible(a, b, eta):
    """eq. (10) for two cells: eta * gap >= sqrt(3) * (smaller side)."""
    d2 = 0
    for (alo, ahi), (blo, bhi) in zip(a.span(), b.span()):
        gap = max(0, blo - ahi, alo - bhi)
        d2 += gap * gap
    side = 1 << (DEPTH_MAX - max(a.depth, b.depth))
    return eta * eta * float(d2) >= 3.0 * float(side * side)


def block_partition(tree, eta=2.0):
    """Return (near, far): near = list of (leaf t, leaf s) with t.leaf_id <=
    s.leaf_id, far = list of (node t, node s) with t.id < s.id."""
    near, far = [], []
    stack = [(tree["root"], tree["root"])]
    while stack:
        t, s = stack.pop()
        if admissible(t, s, eta):
            if t.id < s.id:
                far.append((t, s))
            continue
        if t.is_leaf and s.is_leaf:
            if t.leaf_id <= s.leaf_id:
                near.append((t, s))
            continue
        if t.is_leaf:
            stack.extend((t, c) for c in s.children)
        elif s.is_leaf:
            stack.extend((c, s) for c in t.children)
        elif t.depth < s.depth:
            stack.extend((c, s) for c in t.children)
        elif s.depth < t.depth:
            stack.extend((t, c) for c in s.children)
        else:
            stack.extend((c, d) for c in t.children for d in s.children)
    near.sort(key=lambda p: (p[0].leaf_id, p[1].leaf_id))
    far.sort(key=lambda p: (p[0].id, p[1].id))
    return near, far
