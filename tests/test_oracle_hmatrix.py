"""Pins for the oracle's cluster tree, admissibility split and ACA."""

import numpy as np

from oracle.aca import aca, recompress
from oracle.cluster import admissible, build_tree, block_partition, touch, Node, DEPTH_MAX
from oracle.rwg import build_rwg, edge_midpoints
from workloads import icosphere
from conftest import rel


def test_tree_is_a_partition():
    xyz, tri = icosphere(3)
    rwg = build_rwg(xyz, tri)
    for leaf_max in (16, 64, 200):
        tree = build_tree(edge_midpoints(rwg), leaf_max)
        perm = tree["perm"]
        assert np.array_equal(np.sort(perm), np.arange(rwg["N"]))
        lo = 0
        for nd in tree["leaves"]:
            assert nd.lo == lo and nd.hi - nd.lo <= leaf_max
            assert np.all(np.diff(perm[nd.lo:nd.hi]) > 0)      # RWG order inside a leaf
            lo = nd.hi
        assert lo == rwg["N"]


def test_near_far_cover_every_pair_once():
    xyz, tri = icosphere(3)
    rwg = build_rwg(xyz, tri)
    tree = build_tree(edge_midpoints(rwg), 32)
    near, far = block_partition(tree)
    N = rwg["N"]
    cover = np.zeros((N, N), dtype=np.int32)
    for t, s in near:
        cover[t.lo:t.hi, s.lo:s.hi] += 1
        if t is not s:
            cover[s.lo:s.hi, t.lo:t.hi] += 1
        assert touch(t, s)
    for t, s in far:
        cover[t.lo:t.hi, s.lo:s.hi] += 1
        cover[s.lo:s.hi, t.lo:t.hi] += 1
        assert not touch(t, s)
    assert np.all(cover == 1)


def test_touch_integer_geometry():
    def node(depth, ijk):
        return Node(depth, ijk, np.zeros(0, dtype=np.int64))
    a = node(3, (2, 2, 2))
    assert touch(a, node(3, (3, 3, 3)))          # corner contact
    assert not touch(a, node(3, (4, 2, 2)))      # one cell gap
    assert touch(a, node(2, (1, 1, 1)))          # parent contains it
    assert touch(a, node(4, (6, 4, 4)))          # finer cell on the face
    assert not touch(a, node(4, (7, 4, 4)))
    assert DEPTH_MAX == 21


def _node(depth, ijk):
    return Node(depth, ijk, np.zeros(0, dtype=np.int64))


def test_admissibility_eq10_worked_cases():
    """eq. (10), eta dist >= min(dia), on cells of side 1 (depth 21 units):
    a gap of one side along one axis is dist 1, dia sqrt(3), so the pair is
    admissible iff eta >= sqrt(3); a diagonal gap of (1, 1, 1) sides is
    dist sqrt(3), admissible iff eta >= 1; touching cells never are; a cell
    of side 2 at gap 3 from a unit cell: dist 3, min(dia) sqrt(3),
    admissible iff eta >= 1/sqrt(3)."""
    a = _node(21, (10, 10, 10))
    b = _node(21, (12, 10, 10))
    r3 = np.sqrt(3.0)
    assert not admissible(a, b, 1.73) and admissible(a, b, 1.7321)
    c = _node(21, (12, 12, 12))
    assert not admissible(a, c, 0.999) and admissible(a, c, 1.0)
    assert not any(admissible(a, _node(21, (11, 11, 11)), e) for e in (0.0, 2.0, 1e6))
    d = _node(20, (7, 5, 5))                      # spans [14, 16) x [10, 12) x [10, 12)
    assert not admissible(a, d, 1.0 / r3 - 1e-9) and admissible(a, d, 1.0 / r3 + 1e-9)
    assert not admissible(a, b, 0.0)


def test_admissibility_above_sqrt3_is_no_touch():
    """For any eta >= sqrt(3) eq. (10) is the touch test (gap >= the smaller
    side along some axis when the closed cells do not touch), on random pairs
    of cells at random depths."""
    rng = np.random.default_rng(17)
    for _ in range(4000):
        da, db = rng.integers(2, 6, size=2)
        a = _node(int(da), tuple(int(x) for x in rng.integers(0, 1 << da, 3)))
        b = _node(int(db), tuple(int(x) for x in rng.integers(0, 1 << db, 3)))
        for eta in (1.7320508075688774, 2.0, 9.0):
            assert admissible(a, b, eta) == (not touch(a, b))


def test_small_eta_partition_by_brute_force():
    """eta = 1 (below sqrt(3)): the split still covers every (i, j) once; far
    blocks are admissible, near leaf pairs are not, and some near pairs do
    not touch; eta = 0 leaves no far block (every leaf pair near)."""
    xyz, tri = icosphere(3)
    rwg = build_rwg(xyz, tri)
    tree = build_tree(edge_midpoints(rwg), 32)
    N = rwg["N"]
    near, far = block_partition(tree, 1.0)
    cover = np.zeros((N, N), dtype=np.int32)
    for t, s in near:
        cover[t.lo:t.hi, s.lo:s.hi] += 1
        if t is not s:
            cover[s.lo:s.hi, t.lo:t.hi] += 1
        assert not admissible(t, s, 1.0)
    for t, s in far:
        cover[t.lo:t.hi, s.lo:s.hi] += 1
        cover[s.lo:s.hi, t.lo:t.hi] += 1
        assert admissible(t, s, 1.0)
    assert np.all(cover == 1)
    near2, _ = block_partition(tree, 2.0)
    assert len(near) > len(near2) and any(not touch(t, s) for t, s in near)
    n0, f0 = block_partition(tree, 0.0)
    L = len(tree["leaves"])
    assert not f0 and len(n0) == L * (L + 1) // 2


def test_aca_recovers_exact_low_rank():
    rng = np.random.default_rng(3)
    m, n, r = 60, 45, 4
    A = (rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))) @ \
        (rng.standard_normal((r, n)) + 1j * rng.standard_normal((r, n)))
    U, V = aca(lambda i: A[i], lambda j: A[:, j], lambda: A, m, n, 1e-10)
    assert U.shape[1] == r
    assert rel(U @ V.T, A) < 1e-12


def test_aca_dense_fallback_and_recompress():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    U, V = aca(lambda i: A[i], lambda j: A[:, j], lambda: A, 8, 8, 1e-3)
    assert rel(U @ V.T, A) < 1e-3
    # recompression of an exact rank-2 pair padded with dependent columns
    B = rng.standard_normal((20, 2)) + 0j
    C = rng.standard_normal((15, 2)) + 0j
    U2, V2 = recompress(np.hstack([B, B]), np.hstack([C, C]), 1e-12)
    assert U2.shape[1] == 2 and rel(U2 @ V2.T, 2 * B @ C.T) < 1e-12


def test_hmatrix_vs_dense(c0_hmatrix, c0_dense):
    """||Z - H||_F <= 2 eps ||Z||_F and H x within 2 eps of Z x (eps = 1e-3)."""
    H = c0_hmatrix
    P = H.perm
    Zt = c0_dense[np.ix_(P, P)]
    assert rel(H.dense_near() + H.dense_far(), Zt) <= 2e-3
    x = np.random.default_rng(0).standard_normal((H.N, 3)) + 0j
    assert rel(H.matvec(x), Zt @ x) <= 2e-3
    # near blocks are the exact Galerkin entries
    for (t, s), B in list(H.near.items())[::17]:
        assert np.array_equal(B, Zt[H.group_slice(t), H.group_slice(s)])
    # per block the partial-pivoting stopping rule is a heuristic, so eq. (12)
    # holds only approximately block by block (observed max ~2.1 eps)
    errs = [rel(U @ V.T, Zt[tlo:thi, slo:shi]) for tlo, thi, slo, shi, U, V in H.far[::3]]
    assert max(errs) <= 5e-3 and np.median(errs) <= 1e-3


def test_minimum_box_side_stops_the_tree():
    """Electrically sized leaves: no cell narrower than box_min is created; a
    leaf holds more than leaf_max points only at that depth limit."""
    from oracle.cluster import root_side, depth_limit
    xyz, tri = icosphere(3)
    rwg = build_rwg(xyz, tri)
    pts = edge_midpoints(rwg)
    side = root_side(pts)
    for box_min in (0.3, 0.75, 1.2, 5.0):
        d = depth_limit(side, box_min)
        assert side / 2.0 ** d >= box_min or d == 0
        assert side / 2.0 ** (d + 1) < box_min
        tree = build_tree(pts, 16, box_min)
        assert np.array_equal(np.sort(tree["perm"]), np.arange(rwg["N"]))
        for nd in tree["leaves"]:
            assert nd.depth <= d
            assert nd.hi - nd.lo <= 16 or nd.depth == d
        if box_min >= side:
            assert len(tree["leaves"]) == 1
    # box_min = 0 is the plain count rule
    a, b = build_tree(pts, 16), build_tree(pts, 16, 0.0)
    assert np.array_equal(a["perm"], b["perm"]) and len(a["leaves"]) == len(b["leaves"])


def test_cluster_sample_is_the_principal_sub_hmatrix():
    """build_hmatrix_cluster (the bounded sample the CPU baseline times) is
    the principal sub-H-matrix of one cluster of the full H-matrix: its near
    and far blocks equal the full build's blocks inside the cluster, and its
    dense near + far field equals the full one restricted to the cluster's
    unknowns."""
    from oracle.hmatrix import build_hmatrix, build_hmatrix_cluster
    xyz, tri = icosphere(3, 1.0)
    full = build_hmatrix(xyz, tri, 200e6, 32, 1e-3, workers=4)
    sub, info = build_hmatrix_cluster(xyz, tri, 200e6, 32, 1e-3, 600, workers=4)
    assert info["N"] == full.N and len(info["leaf_sizes"]) == full.M
    assert 0 < sub.N <= 600
    idx = sub.rwg_index
    pos = {int(r): p for p, r in enumerate(full.perm)}
    lo = pos[int(idx[0])]
    assert [pos[int(r)] for r in idx] == list(range(lo, lo + sub.N))     # one contiguous tree range
    Zf = full.dense_near() + full.dense_far()
    Zs = sub.dense_near() + sub.dense_far()
    assert np.array_equal(Zs, Zf[lo:lo + sub.N, lo:lo + sub.N])
