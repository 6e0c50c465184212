"""Pins for the oracle's Schur scaling (eqs. 14-23) and power series
(eqs. 24-36): the 4-block worked example, block-diagonality, transposed left
coefficients, the closed form, dense LU special cases, order independence and
reciprocity."""

import numpy as np
import pytest

from oracle.hmatrix import HMatrix
from oracle.planewave import excitation
from oracle.scaling import (SingularBlock, group_graph, min_degree_order, natural_order,
                            schur_scaling)
from oracle.series import PowerSeries, dense_two_term
from conftest import rel


def _rand_sym(rng, n):
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return A + A.T + 4 * n * np.eye(n)


def _four_block():
    """eq. (14): four groups, block (1,4) far (zero in Z_N)."""
    rng = np.random.default_rng(7)
    sizes = [3, 4, 2, 5]
    lo = np.cumsum([0] + sizes)
    groups = np.stack([lo[:-1], lo[1:]], 1)
    near = {}
    for i in range(4):
        near[(i, i)] = _rand_sym(rng, sizes[i])
        for j in range(i + 1, 4):
            if (i, j) != (0, 3):
                near[(i, j)] = rng.standard_normal((sizes[i], sizes[j])) + 1j * rng.standard_normal((sizes[i], sizes[j]))
    return HMatrix(sum(sizes), np.arange(sum(sizes)), groups, near, [])


def test_worked_example_step_one():
    """After the first scaling step the blocks are those of eq. (21)."""
    H = _four_block()
    Z = H.dense_near()
    sl = [H.group_slice(g) for g in range(4)]
    blk = lambda M, i, j: M[sl[i], sl[j]]
    # alpha_1 and alpha'_1 of eqs. (16), (18), built densely
    inv11 = np.linalg.inv(blk(Z, 0, 0))
    a1 = np.eye(H.N, dtype=complex)
    a1l = np.eye(H.N, dtype=complex)
    for j in (1, 2):
        a1[sl[0], sl[j]] = -inv11 @ blk(Z, 0, j)
        a1l[sl[j], sl[0]] = -blk(Z, j, 0) @ inv11
    Z1 = a1l @ Z @ a1                                         # eq. (20)
    for j in (1, 2):
        assert np.abs(blk(Z1, 0, j)).max() < 1e-13 and np.abs(blk(Z1, j, 0)).max() < 1e-13
        for k in (1, 2):
            ref = blk(Z, j, k) - blk(Z, j, 0) @ inv11 @ blk(Z, 0, k)
            assert rel(blk(Z1, j, k), ref) < 1e-13
    for (j, k) in ((1, 3), (2, 3), (3, 3), (3, 1)):         # untouched by step 1
        assert np.array_equal(blk(Z1, j, k), blk(Z, j, k))
    # the oracle's first step produces the same coefficients
    S = schur_scaling(H, [0, 1, 2, 3])
    assert S.later[0] == [1, 2]
    for j in (1, 2):
        assert rel(-S.C[(0, j)], a1[sl[0], sl[j]]) < 1e-14
        # left coefficient = transpose of the right one (symmetric Z_N)
        assert rel(a1l[sl[j], sl[0]], a1[sl[0], sl[j]].T) < 1e-13


def _alpha_product(H, S):
    A = np.eye(H.N, dtype=complex)
    for i in S.order:
        ai = np.eye(H.N, dtype=complex)
        for j in S.later[i]:
            ai[H.group_slice(i), H.group_slice(j)] = -S.C[(i, j)]
        A = A @ ai
    return A


@pytest.mark.parametrize("order_kind", ["natural", "mindeg"])
def test_block_diagonal_after_all_steps(order_kind):
    """eq. (23): A^T Z_N A is block diagonal with blocks D_i, incl. fill-in."""
    H = _four_block()
    order = natural_order(4) if order_kind == "natural" else min_degree_order(group_graph(H))
    S = schur_scaling(H, order)
    Z = H.dense_near()
    A = _alpha_product(H, S)
    T = A.T @ Z @ A
    for i in range(4):
        for j in range(4):
            b = T[H.group_slice(i), H.group_slice(j)]
            if i == j:
                assert rel(b, S.D[i]) < 1e-13
            else:
                assert np.abs(b).max() < 1e-12 * np.abs(Z).max()
    # fill-in: groups 1 and 4 are both coupled to 2 and 3; the block (1,4) is
    # created when a common neighbour is eliminated first
    if order_kind == "natural":
        assert S.later[1] == [2, 3] and S.later[2] == [3]


def test_fill_in_created_and_symmetric(small_sphere):
    H = small_sphere
    S = schur_scaling(H, natural_order(H.M))
    n_coupled = sum(len(v) for v in group_graph(H).values()) // 2
    assert sum(len(v) for v in S.later.values()) > n_coupled      # fill-in exists
    for g, D in S.D.items():                                      # Schur blocks stay symmetric
        assert np.abs(D - D.T).max() <= 1e-13 * np.abs(D).max()


def test_closed_form_two_terms(small_sphere, c0_hmatrix, c0_workload):
    """x2 = y - Z_N^{-1} Z_F y, y = Z_N^{-1} b, by dense LU (any order)."""
    for H in (small_sphere, c0_hmatrix):
        b = excitation(H.rwg, H.op.freq_hz, [[0, 0, -1.0], [0.6, 0, -0.8]], [[1.0, 0, 0], [0.8, 0, 0.6]])
        bt = H.to_tree(b)
        ref = dense_two_term(H.dense_near(), H.dense_far(), bt, 2)
        for order in (natural_order(H.M), min_degree_order(group_graph(H))):
            x, ratio = PowerSeries(H, schur_scaling(H, order)).solve(bt, 2)
            assert rel(x, ref) < 1e-11
            assert ratio.shape == (1, 2)
        x1, _ = PowerSeries(H, schur_scaling(H, natural_order(H.M))).solve(bt, 1)
        assert rel(x1, np.linalg.solve(H.dense_near(), bt)) < 1e-11


def test_no_far_field_is_direct_solve(c0_workload):
    """With nothing admissible (Z_F = 0) the series is the dense LU solution
    of the full MoM system."""
    from oracle.hmatrix import build_hmatrix
    from workloads import icosphere
    xyz, tri = icosphere(2)
    H = build_hmatrix(xyz, tri, 300e6, 32, 1e-3, eta_far=False, workers=4)
    b = excitation(H.rwg, 300e6, [[0, 0, -1.0]], [[1.0, 0, 0]])
    x, _ = PowerSeries(H, schur_scaling(H, min_degree_order(group_graph(H)))).solve_rwg(b, 2)
    ref = np.linalg.solve(H.op.dense(), b)
    assert rel(x, ref) < 1e-12


def test_series_converges_to_lu_when_contractive(small_sphere):
    """With the far field scaled down so that the series converges, many
    terms reproduce the dense LU solution of Z_N + Z_F."""
    H0 = small_sphere
    far = [(a, b, c, d, 0.02 * U, V) for a, b, c, d, U, V in H0.far]
    H = HMatrix(H0.N, H0.perm, H0.groups, H0.near, far)
    b = H.to_tree(excitation(H0.rwg, 300e6, [[0, 0, -1.0]], [[1.0, 0, 0]]))
    ps = PowerSeries(H, schur_scaling(H, min_degree_order(group_graph(H))))
    x, ratios = ps.solve(b, 40)
    assert np.all(ratios[:, 0] < 0.9)
    assert rel(x, np.linalg.solve(H.dense_near() + H.dense_far(), b)) < 1e-10


def test_reciprocity(c0_hmatrix):
    """P = (I - K) Z_N^{-1} is complex symmetric, so B^T X is symmetric."""
    H = c0_hmatrix
    th = np.deg2rad([0.0, 40.0, 95.0, 150.0])
    khat = -np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    pol = np.stack([np.cos(th), 0 * th, -np.sin(th)], 1)
    B = excitation(H.rwg, H.op.freq_hz, khat, pol)
    X, _ = PowerSeries(H, schur_scaling(H, natural_order(H.M))).solve_rwg(B, 2)
    G = B.T @ X
    assert np.abs(G - G.T).max() < 1e-12 * np.abs(G).max()


def test_singular_block_detected():
    H = _four_block()
    near = dict(H.near)
    near[(2, 2)] = np.zeros_like(near[(2, 2)])
    near[(0, 2)] = np.zeros_like(near[(0, 2)])
    near[(1, 2)] = np.zeros_like(near[(1, 2)])
    near[(2, 3)] = np.zeros_like(near[(2, 3)])
    with pytest.raises(SingularBlock):
        schur_scaling(HMatrix(H.N, H.perm, H.groups, near, []), [0, 1, 2, 3])


def test_pivot_threshold_two_by_two():
    """Numerical singularity = an LU pivot below n eps max|Z|.  For a 2 x 2
    block with |a| >= |c| partial pivoting keeps row 0, and the pivots are a
    and d - c b / a in closed form: a second pivot of half the threshold is
    singular, twice the threshold is not."""
    from oracle.scaling import pivots_ok
    a, b, c = 4.0 + 1.0j, 1.0 - 2.0j, 2.0 + 0.5j
    thr = 2 * 2.0 ** -52 * abs(a)              # max |Z| = |a| here
    for t, ok in ((0.5, False), (2.0, True)):
        d = c * b / a + t * thr
        Z = np.array([[a, b], [c, d]])
        assert np.max(np.abs(Z)) == abs(a)
        assert pivots_ok(Z) is ok


def test_pivot_threshold_known_lu():
    """A = L U with |L_ij| < 1 keeps its row order under partial pivoting, so
    its pivots are diag(U): a pivot of 1e-20 max|A| is flagged, 1e-8 is not."""
    from oracle.scaling import pivots_ok
    rng = np.random.default_rng(3)
    n = 6
    L = np.tril(0.4 * (rng.uniform(-1, 1, (n, n)) + 1j * rng.uniform(-1, 1, (n, n))), -1) + np.eye(n)
    U = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), 1)
    for small, ok in ((1e-20, False), (1e-8, True)):
        d = np.full(n, 3.0 + 0.0j)
        d[4] = small
        A = L @ (U + np.diag(d))
        assert pivots_ok(A) is ok


def test_near_singular_block_detected():
    """A symmetric diagonal block whose rows 0 and 1 differ in one entry by
    1e-18 of the block's size is numerically singular: the elimination stops
    with an error (the exactly singular case is test_singular_block_detected)."""
    H = _four_block()
    near = dict(H.near)
    B = near[(0, 0)].copy()
    B[0, 1] = B[1, 0] = B[0, 0]
    B[1, 2] = B[2, 1] = B[0, 2]
    B[1, 1] = B[0, 0] + 1e-18 * np.abs(B).max()
    assert np.array_equal(B, B.T)
    near[(0, 0)] = B
    with pytest.raises(SingularBlock):
        schur_scaling(HMatrix(H.N, H.perm, H.groups, near, []), [0, 1, 2, 3])
    # the untouched matrix factors without complaint
    schur_scaling(H, [0, 1, 2, 3])
