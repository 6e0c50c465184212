"""GPU parity of the HIP hot path against the CPU oracle (through the C ABI).

The oracle's own H-matrix is installed in the library with hps_set_hmatrix,
so both sides start from the same Z_N and Z_F; the library then runs its
symbolic phase (nested-dissection order, different from the oracle's minimum
degree), the device setup and the power-series solve.  The two-term result
does not depend on the order, so the comparison is element by element.

Bars: FP64 throughout, so currents agree to 1e-10 relative per RHS (rounding
of two different elimination orders, amplified by the conditioning of the
near-field blocks), the eq. (45) ratio to 1e-9 and the RCS to 1e-6 dB -- far
inside the 1e-3 current / 0.1 dB target.
"""

import math

import numpy as np
import pytest

from oracle.hmatrix import HMatrix, build_hmatrix
from oracle.planewave import excitation, monostatic_rcs
from oracle.scaling import SingularBlock, group_graph, min_degree_order, natural_order, schur_scaling
from oracle.series import PowerSeries
from workloads import icosphere, monostatic_angles
from hmat_io import hmatrix_arrays, per_rhs_rel
from conftest import rel

torch = pytest.importorskip("torch")
from paper_2109_04129_amd import hps  # noqa: E402

pytestmark = pytest.mark.gpu


def _ctx():
    assert torch.cuda.is_available(), "the GPU tests need a HIP device"
    return hps.hps_create(0, torch.cuda.current_stream().cuda_stream)


def _install(ctx, H, xyz, tri, freq, terms=2, leaf=128, ordering=0, open_surface=False):
    (hps.hps_set_open_mesh if open_surface else hps.hps_set_mesh)(ctx, xyz, tri)
    p = hps.hps_params_default(freq_hz=freq, leaf_max=leaf, aca_tol=1e-3, terms=terms, ordering=ordering)
    a = hmatrix_arrays(H)
    hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"],
                        a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
    hps.hps_setup(ctx)


def _solve(ctx, N, khat, pol):
    R = len(khat)
    X = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
    st, rcs, ratio = hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
    torch.cuda.synchronize()
    return st, X.cpu().numpy().T.copy(), rcs, ratio


def _oracle(H, freq, khat, pol, terms, order="mindeg"):
    b = excitation(H.rwg, freq, khat, pol)
    o = min_degree_order(group_graph(H)) if order == "mindeg" else natural_order(H.M)
    x, ratios = PowerSeries(H, schur_scaling(H, o)).solve_rwg(b, terms)
    sig = monostatic_rcs(H.rwg, freq, khat, pol, x)
    return x, ratios, sig


@pytest.fixture(scope="module")
def small():
    xyz, tri = icosphere(2, 1.0)
    H = build_hmatrix(xyz, tri, 300e6, 16, 1e-3, workers=8)
    return xyz, tri, H


@pytest.mark.parametrize("ordering", [0, 1])
def test_sphere_1920_two_terms(c0_workload, c0_hmatrix, ordering):
    """Nested-dissection order on the GPU vs minimum degree in the oracle
    (currents and RCS are order-independent); with the natural order on both
    sides the eq. (45) ratio, which lives in the scaled unknowns, agrees too."""
    w, H = c0_workload, c0_hmatrix
    print("case: sphere 1,920 unknowns, oracle H-matrix, T=2, ordering", ordering, flush=True)
    khat, pol = monostatic_angles([0.0, 33.0, 90.0, 147.0, 180.0], [0.0, 10.0, 0.0, 200.0, 0.0])
    khat = np.vstack([w["khat"], khat])
    pol = np.vstack([w["pol"], pol])
    ctx = _ctx()
    try:
        _install(ctx, H, w["xyz"], w["tri"], w["freq_hz"], terms=2, ordering=ordering)
        st, X, rcs, ratio = _solve(ctx, H.N, khat, pol)
        x, ratios, sig = _oracle(H, w["freq_hz"], khat, pol, 2, order="mindeg" if ordering == 0 else "natural")
        err = per_rhs_rel(X, x)
        print("max rel current err", err.max(), "ratio", ratio, flush=True)
        assert err.max() < 1e-10
        assert np.max(np.abs(10 * np.log10(rcs / sig))) < 1e-6
        if ordering == 1:
            assert np.allclose(ratio, ratios[0], rtol=1e-9)
        assert st == (hps.HPS_WRATIO if np.any(ratio >= 0.1) else hps.HPS_OK)
    finally:
        hps.hps_destroy(ctx)


def test_leaves_of_256(c0_workload):
    """Oracle H-matrix with leaves of up to 256 unknowns (oracle pivots = those
    groups); the library cuts them into pivots of at most 128.  Currents and
    RCS do not depend on the blocking of the elimination."""
    w = c0_workload
    H = build_hmatrix(w["xyz"], w["tri"], w["freq_hz"], 256, w["aca_tol"], workers=8)
    sizes = H.groups[:, 1] - H.groups[:, 0]
    print("case: sphere 1,920 unknowns, leaves <= 256 (max %d), T=2" % sizes.max(), flush=True)
    assert sizes.max() > 128
    khat, pol = monostatic_angles([0.0, 60.0, 120.0], [0.0, 30.0, 90.0])
    ctx = _ctx()
    try:
        _install(ctx, H, w["xyz"], w["tri"], w["freq_hz"], terms=2, leaf=256)
        st, X, rcs, ratio = _solve(ctx, H.N, khat, pol)
        x, ratios, sig = _oracle(H, w["freq_hz"], khat, pol, 2)
        err = per_rhs_rel(X, x)
        print("max rel current err", err.max(), flush=True)
        assert err.max() < 1e-10
        assert np.max(np.abs(10 * np.log10(rcs / sig))) < 1e-6
    finally:
        hps.hps_destroy(ctx)


@pytest.mark.parametrize("terms", [1, 2, 3])
def test_small_sphere_ragged_rhs(small, terms):
    """480 unknowns in 56 groups of 1..16, 37 RHS (ragged RHS tiles)."""
    xyz, tri, H = small
    print("case: sphere 480 unknowns, R=37, T=%d" % terms, flush=True)
    th = np.linspace(0.0, 180.0, 37)
    khat, pol = monostatic_angles(th, 0.5 * th)
    ctx = _ctx()
    try:
        _install(ctx, H, xyz, tri, 300e6, terms=terms, leaf=16, ordering=1)
        st, X, rcs, ratio = _solve(ctx, H.N, khat, pol)
        x, ratios, sig = _oracle(H, 300e6, khat, pol, terms, order="natural")
        assert per_rhs_rel(X, x).max() < 1e-10
        assert np.max(np.abs(10 * np.log10(rcs / sig))) < 1e-6
        if terms > 1:
            assert np.allclose(ratio, ratios[0], rtol=1e-9)
    finally:
        hps.hps_destroy(ctx)


def test_hmatvec_excitation_and_arbitrary_rhs(small):
    xyz, tri, H = small
    print("case: hmatvec / excitation / solve_rhs on 480 unknowns", flush=True)
    rng = np.random.default_rng(5)
    R = 3
    Xh = rng.standard_normal((H.N, R)) + 1j * rng.standard_normal((H.N, R))
    ctx = _ctx()
    try:
        _install(ctx, H, xyz, tri, 300e6, terms=2, leaf=16, ordering=1)
        Xd = torch.from_numpy(np.ascontiguousarray(Xh.T)).cuda()
        Yd = torch.zeros_like(Xd)
        hps.hps_hmatvec(ctx, R, Xd.data_ptr(), Yd.data_ptr())
        torch.cuda.synchronize()
        ref = H.to_rwg(H.matvec(H.to_tree(Xh)))
        assert per_rhs_rel(Yd.cpu().numpy().T, ref).max() < 1e-13
        khat, pol = monostatic_angles([10.0, 80.0], [0.0, 45.0])
        Bd = torch.zeros((2, H.N), dtype=torch.complex128, device="cuda")
        hps.hps_excitation(ctx, khat, pol, Bd.data_ptr())
        torch.cuda.synchronize()
        bref = excitation(H.rwg, 300e6, khat, pol)
        assert per_rhs_rel(Bd.cpu().numpy().T, bref).max() < 1e-13
        Xo = torch.zeros_like(Xd)
        st, ratio = hps.hps_solve_rhs(ctx, R, Xd.data_ptr(), Xo.data_ptr())
        torch.cuda.synchronize()
        xo, ratios = PowerSeries(H, schur_scaling(H, natural_order(H.M))).solve_rwg(Xh, 2)
        assert per_rhs_rel(Xo.cpu().numpy().T, xo).max() < 1e-10
        assert np.allclose(ratio, ratios[0], rtol=1e-9)
    finally:
        hps.hps_destroy(ctx)


def test_singular_block_reported(small):
    """A zero scaled diagonal block must come back as HPS_ESINGULAR."""
    xyz, tri, H0 = small
    near = {k: v.copy() for k, v in H0.near.items()}
    for (t, s) in near:
        if t == 0 or s == 0:
            near[(t, s)][:] = 0.0
    H = HMatrix(H0.N, H0.perm, H0.groups, near, H0.far)
    ctx = _ctx()
    try:
        with pytest.raises(hps.HpsError) as ei:
            _install(ctx, H, xyz, tri, 300e6, leaf=16)
        assert ei.value.status == -4
    finally:
        hps.hps_destroy(ctx)


def test_near_singular_block_reported(small):
    """A scaled diagonal block that is singular to working precision (rows 0
    and 1 of group 0 differ in one entry by 1e-18 of the block's size; the
    natural order eliminates group 0 first, so Z~_00 = Z_00) comes back as
    HPS_ESINGULAR: its LU pivot falls below n eps max|D_ij|, as in the oracle."""
    xyz, tri, H0 = small
    near = {k: v.copy() for k, v in H0.near.items()}
    B = near[(0, 0)]
    n = B.shape[0]
    B[0, 1] = B[1, 0] = B[0, 0]
    for j in range(2, n):
        B[1, j] = B[j, 1] = B[0, j]
    B[1, 1] = B[0, 0] + 1e-18 * np.abs(B).max()
    H = HMatrix(H0.N, H0.perm, H0.groups, near, H0.far)
    print("case: near-singular diagonal block of group 0 (%d unknowns), natural order" % n, flush=True)
    with pytest.raises(SingularBlock):
        schur_scaling(H, natural_order(H.M))
    ctx = _ctx()
    try:
        with pytest.raises(hps.HpsError) as ei:
            _install(ctx, H, xyz, tri, 300e6, leaf=16, ordering=1)
        assert ei.value.status == -4
    finally:
        hps.hps_destroy(ctx)


BF16_TWO_TERM = pytest.mark.xfail(
    strict=True, reason="BF16 far factors without the residual pass: measured 2.7e-3 against 1e-3 (the two-term "
                        "series carries the 2^-9 unit roundoff of BF16 unreduced); one FP32 residual pass meets 1e-3")


@pytest.mark.parametrize("precision,refine,bar", [(2, 0, 1e-3), (2, 1, 1e-3),
                                                  pytest.param(1, 0, 1e-3, marks=BF16_TWO_TERM), (1, 1, 1e-3)])
def test_precision_form(c0_workload, c0_hmatrix, precision, refine, bar):
    """Precision form (FP32 solve on MFMA, 16-bit far factors with per-block
    FP32 scale, optional FP32 residual pass) against the FP64 oracle at the
    matching number of terms: one residual pass with the two-term operator P
    gives x + P(b - Hx) = (I - K + K^2 - K^3) Z_N^-1 b, the four-term series.
    Every case is held to the 1e-3 / 0.1 dB target.  With one pass (FP32 far
    factors in the residual and its correction) both 16-bit formats meet it.
    The two-term series alone carries the far-factor rounding unreduced: FP16
    (unit roundoff 2^-12) meets it, BF16 (2^-9) does not (an expected
    failure, with the measured error)."""
    w, H = c0_workload, c0_hmatrix
    print("case: sphere 1,920, precision %d, refine %d" % (precision, refine), flush=True)
    khat, pol = monostatic_angles(np.linspace(0.0, 180.0, 7), np.zeros(7))
    ctx = _ctx()
    try:
        hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
        p = hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=64, aca_tol=1e-3, terms=2, ordering=1,
                                   precision=precision, refine_passes=refine)
        a = hmatrix_arrays(H)
        hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"],
                            a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        hps.hps_setup(ctx)
        st, X, rcs, ratio = _solve(ctx, H.N, khat, pol)
    finally:
        hps.hps_destroy(ctx)
    x, ratios, sig = _oracle(H, w["freq_hz"], khat, pol, 4 if refine else 2, order="natural")
    err = per_rhs_rel(X, x).max()
    db = np.max(np.abs(10 * np.log10(rcs / sig)))
    print("precision %d refine %d: max rel current err %.3e, max RCS err %.4f dB" % (precision, refine, err, db))
    assert err < bar
    assert db < 0.1
    assert np.allclose(ratio, ratios[0], rtol=1e-2)


@pytest.mark.parametrize("precision,bar", [(0, 1e-9), (2, 1e-4)])
def test_adaptive_series_reaches_the_direct_solution(small, precision, bar):
    """With the far field scaled by 0.1 the series contracts; the adaptive
    term count (series_tol) runs it until ||it_t|| / ||it_0|| < 1e-11 and the
    currents equal the direct solution of (Z_N + 0.1 Z_F) x = b (dense LU of
    the oracle's blocks), which the series converges to (eqs. 27-36)."""
    xyz, tri, H = small
    a = hmatrix_arrays(H)
    c = 0.1
    a["far_uv"] = a["far_uv"] * np.sqrt(c)           # U and V scaled: every far block times c
    khat, pol = monostatic_angles([0.0, 75.0, 160.0], [0.0, 40.0, 250.0])
    b = excitation(H.rwg, 300e6, khat, pol)
    Z = H.dense_near() + c * H.dense_far()           # tree order
    P = H.perm
    xt = np.linalg.solve(Z, b[P])
    x = np.empty_like(xt)
    x[P] = xt
    print("case: small sphere, far field x 0.1, adaptive series, precision", precision, flush=True)
    ctx = _ctx()
    try:
        hps.hps_set_mesh(ctx, xyz, tri)
        p = hps.hps_params_default(freq_hz=300e6, leaf_max=16, aca_tol=1e-3, terms=80, series_tol=1e-11,
                                   precision=precision, refine_passes=1 if precision else 0)
        hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"],
                            a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        hps.hps_setup(ctx)
        st, X, rcs, ratio = _solve(ctx, H.N, khat, pol)
        used = hps.hps_stats(ctx)["device"]["terms_used"]
    finally:
        hps.hps_destroy(ctx)
    err = per_rhs_rel(X, x)
    print("terms used", used, "max rel err vs direct", err.max(), "ratio", ratio, flush=True)
    assert 2 < used < 80
    assert err.max() < bar


def test_half_wavelength_leaves():
    """Electrically sized leaves (cells of at least half a wavelength, Sec.
    V.A) on the 1,920-unknown sphere at 600 MHz (leaf_max 64 would split
    further): library vs oracle on the oracle's H-matrix, currents and RCS
    to the parity bar (the library's own build with the same rule matches
    the oracle's, checked on the CPU)."""
    xyz, tri = icosphere(3, 1.0)
    f = 600e6
    lam = 299792458.0 / f
    H = build_hmatrix(xyz, tri, f, 16, 1e-3, workers=8, box_min=0.5 * lam)
    sizes = H.groups[:, 1] - H.groups[:, 0]
    print("case: sphere 1,920 unknowns at 600 MHz, leaves >= lambda/2 (%d groups, max %d, %d far blocks)"
          % (H.M, sizes.max(), len(H.far)), flush=True)
    assert len(H.far) > 0 and sizes.max() > 16
    khat, pol = monostatic_angles([0.0, 90.0], [0.0, 0.0])
    ctx = _ctx()
    try:
        _install(ctx, H, xyz, tri, f, terms=2, leaf=16)
        st, X, rcs, ratio = _solve(ctx, H.N, khat, pol)
    finally:
        hps.hps_destroy(ctx)
    x, _, sig = _oracle(H, f, khat, pol, 2)
    err = per_rhs_rel(X, x)
    print("max rel current err", err.max(), "ratio", ratio, flush=True)
    assert err.max() < 1e-10
    assert np.max(np.abs(10 * np.log10(rcs / sig))) < 1e-6


def test_open_plate():
    """The square plate of Sec. V.C.2 at 2 wavelengths (1,160 unknowns, open
    surface, EFIE): GPU vs oracle on the oracle's H-matrix, theta = 0..180."""
    from workloads import workload
    w = workload("plate_2lambda_300MHz")
    H = build_hmatrix(w["xyz"], w["tri"], w["freq_hz"], w["leaf_max"], w["aca_tol"], workers=8, open_surface=True)
    print("case: plate 2 lambda, 1,160 unknowns, %d RHS" % len(w["khat"]), flush=True)
    ctx = _ctx()
    try:
        _install(ctx, H, w["xyz"], w["tri"], w["freq_hz"], terms=2, leaf=w["leaf_max"], open_surface=True)
        st, X, rcs, ratio = _solve(ctx, H.N, w["khat"], w["pol"])
    finally:
        hps.hps_destroy(ctx)
    x, _, sig = _oracle(H, w["freq_hz"], w["khat"], w["pol"], 2)
    err = per_rhs_rel(X, x)
    print("max rel current err", err.max(), "ratio", ratio, flush=True)
    assert err.max() < 1e-10
    assert np.max(np.abs(10 * np.log10(rcs / sig))) < 1e-6


def test_device_hmatrix_build(c0_workload, c0_hmatrix, c0_dense):
    """hps_build_hmatrix on a device context computes the near blocks, the
    ACA samples of the far blocks and their recompression on the GPU (Gram
    matrices and recompressed factors on the device, k x k eigenproblems on
    host threads): near entries equal the oracle's and the host build's
    (host_near = 1: QR + SVD recompression on the host) to rounding; the far
    field approximates the dense matrix to the ACA bound (2 eps), like the
    host build, with the same structure and mean rank within 10%."""
    w, H = c0_workload, c0_hmatrix
    print("case: sphere 1,920 unknowns, H-matrix build on the device", flush=True)
    out = {}
    for host_near in (0, 1):
        ctx = _ctx()
        try:
            hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
            hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"],
                                                              aca_tol=w["aca_tol"], host_near=host_near))
            out[host_near] = hps.hps_get_hmatrix(ctx)
        finally:
            hps.hps_destroy(ctx)
    G, C = out[0], out[1]
    assert np.array_equal(G["near_ts"], C["near_ts"]) and np.array_equal(G["far_rng"], C["far_rng"])
    keys = [tuple(x) for x in G["near_ts"].reshape(-1, 2)]
    assert keys == sorted(H.near)
    worst_o, worst_h = 0.0, 0.0
    for b, k in enumerate(keys):
        blk = G["near_vals"][G["near_off"][b]:G["near_off"][b + 1]].reshape(H.near[k].shape)
        hst = C["near_vals"][C["near_off"][b]:C["near_off"][b + 1]].reshape(H.near[k].shape)
        scale = np.abs(H.near[k]).max()
        worst_o = max(worst_o, np.abs(blk - H.near[k]).max() / scale)
        worst_h = max(worst_h, np.abs(blk - hst).max() / scale)
    P = H.perm
    Zt = c0_dense[np.ix_(P, P)]
    errs = {}
    for name, L in (("device", G), ("host", C)):
        Zh = H.dense_near()
        for b, (tlo, thi, slo, shi) in enumerate(L["far_rng"].reshape(-1, 4)):
            r, m, n = L["far_rank"][b], thi - tlo, shi - slo
            uv = L["far_uv"][L["far_off"][b]:L["far_off"][b + 1]]
            B = uv[:m * r].reshape(r, m).T @ uv[m * r:].reshape(r, n)
            Zh[tlo:thi, slo:shi] = B
            Zh[slo:shi, tlo:thi] = B.T
        errs[name] = rel(Zh, Zt)
    print("device near vs oracle %.2e, vs host %.2e; far-field error device %.2e host %.2e; mean rank %.2f / %.2f"
          % (worst_o, worst_h, errs["device"], errs["host"], G["far_rank"].mean(), C["far_rank"].mean()), flush=True)
    assert worst_o <= 1e-12 and worst_h <= 1e-12
    assert errs["device"] <= 2e-3 and errs["host"] <= 2e-3
    assert abs(G["far_rank"].mean() - C["far_rank"].mean()) <= 0.1 * C["far_rank"].mean()

def test_exported_hmatrix_solves_identically(small, tmp_path):
    """An H-matrix written by hps_export_hmatrix and read back by
    hps_import_hmatrix into a fresh device context gives the same setup and
    solve, bit for bit, as the context it came from; the library's RWG table
    names the unknowns of the currents."""
    xyz, tri, H = small
    print("case: export / import of a 480-unknown H-matrix, device contexts", flush=True)
    khat, pol = monostatic_angles([0.0, 60.0, 135.0], [0.0, 90.0, 200.0])
    path = str(tmp_path / "small.hmat")
    a = _ctx()
    try:
        _install(a, H, xyz, tri, 300e6, leaf=16)
        hps.hps_export_hmatrix(a, path)
        _, Xa, rcs_a, rat_a = _solve(a, H.N, khat, pol)
        ev, _, _ = hps.hps_rwg(a)
    finally:
        hps.hps_destroy(a)
    b = _ctx()
    try:
        hps.hps_set_mesh(b, xyz, tri)
        hps.hps_import_hmatrix(b, path)
        hps.hps_setup(b)
        _, Xb, rcs_b, rat_b = _solve(b, H.N, khat, pol)
    finally:
        hps.hps_destroy(b)
    assert np.array_equal(Xa, Xb) and np.array_equal(rcs_a, rcs_b) and np.array_equal(rat_a, rat_b)
    assert np.array_equal(ev, H.rwg["edges"])


def test_host_pointers_equal_device_pointers(small):
    """X, B and Y may be host memory (found with hipPointerGetAttributes and
    staged through the context's buffers): plane-wave currents, arbitrary-RHS
    solves, excitation and H-matvec give bit for bit the device-pointer
    results."""
    xyz, tri, H = small
    print("case: host vs device pointers, 480 unknowns", flush=True)
    khat, pol = monostatic_angles([0.0, 45.0, 120.0], [0.0, 30.0, 300.0])
    R = len(khat)
    rng = np.random.default_rng(9)
    Bh = np.ascontiguousarray(rng.standard_normal((R, H.N)) + 1j * rng.standard_normal((R, H.N)))
    ctx = _ctx()
    try:
        _install(ctx, H, xyz, tri, 300e6, leaf=16)
        Xd = torch.zeros((R, H.N), dtype=torch.complex128, device="cuda")
        hps.hps_solve_planewaves(ctx, khat, pol, Xd.data_ptr())
        Xh = np.zeros((R, H.N), dtype=np.complex128)
        hps.hps_solve_planewaves(ctx, khat, pol, Xh.ctypes.data)
        torch.cuda.synchronize()
        assert np.array_equal(Xd.cpu().numpy(), Xh)
        Bd = torch.from_numpy(Bh).cuda()
        Yd = torch.zeros_like(Bd)
        hps.hps_solve_rhs(ctx, R, Bd.data_ptr(), Yd.data_ptr())
        Yh = np.zeros_like(Bh)
        hps.hps_solve_rhs(ctx, R, Bh.ctypes.data, Yh.ctypes.data)
        torch.cuda.synchronize()
        assert np.array_equal(Yd.cpu().numpy(), Yh)
        hps.hps_hmatvec(ctx, R, Bd.data_ptr(), Yd.data_ptr())
        hps.hps_hmatvec(ctx, R, Bh.ctypes.data, Yh.ctypes.data)
        torch.cuda.synchronize()
        assert np.array_equal(Yd.cpu().numpy(), Yh)
        hps.hps_excitation(ctx, khat, pol, Yd.data_ptr())
        hps.hps_excitation(ctx, khat, pol, Yh.ctypes.data)
        torch.cuda.synchronize()
        assert np.array_equal(Yd.cpu().numpy(), Yh)
    finally:
        hps.hps_destroy(ctx)


def test_device_mem_cap_on_device(small):
    """A cap below the plan's device memory fails hps_setup with HPS_ENOMEM and
    leaves the context usable: the same H-matrix with the cap lifted sets up
    and solves."""
    xyz, tri, H = small
    print("case: device_mem_cap on a device context", flush=True)
    a = hmatrix_arrays(H)
    ctx = _ctx()
    try:
        hps.hps_set_mesh(ctx, xyz, tri)
        # the H-matrix itself fits (hps_set_hmatrix checks that), the setup plan not
        cap_h = (a["near_vals"].size + a["far_uv"].size) * 16 + H.N * 14 * 10 * 8 + 1024
        for cap, status in ((cap_h, -2), (0, 0)):
            p = hps.hps_params_default(freq_hz=300e6, leaf_max=16, device_mem_cap=cap)
            hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"],
                                a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
            if status:
                with pytest.raises(hps.HpsError) as e:
                    hps.hps_setup(ctx)
                assert e.value.status == status
            else:
                hps.hps_setup(ctx)
                st, X, rcs, ratio = _solve(ctx, H.N, *monostatic_angles([30.0], [0.0]))
                assert np.all(np.isfinite(X))
    finally:
        hps.hps_destroy(ctx)
