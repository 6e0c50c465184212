"""GPU parity of the CFIE variant (eq. 8, not symmetric: separate left
coefficients, eq. 18) against the oracle, through the C ABI.

* the oracle's CFIE H-matrix installed in the library: currents, RCS and
  (natural order on both sides) eq. (45) ratios against the oracle's
  two-term series, at the EFIE parity bars;
* the CFIE excitation against the oracle's;
* the library's own CFIE H-matrix (device near blocks and ACA, host
  recompression) against the dense oracle matrix, and the device-built one
  against the host-built one;
* the precision form against the FP64 four-term series (1e-3);
* a batch of two CFIE problems against single contexts (bitwise);
* random right-hand sides against the oracle, graph replays against eager
  launches (bitwise);
* the converged series (adaptive, many terms) against the Mie series on a
  sphere: the CFIE's series contracts where the EFIE's does not.
"""

import math

import numpy as np
import pytest

from oracle import mie
from oracle.constants import wavenumber
from oracle.hmatrix import build_hmatrix
from oracle.planewave import excitation_cfie, monostatic_rcs
from oracle.scaling import group_graph, min_degree_order, natural_order, schur_scaling
from oracle.series import PowerSeries
from workloads import ellipsoid_mesh, icosphere, monostatic_angles
from hmat_io import hmatrix_arrays, per_rhs_rel

torch = pytest.importorskip("torch")
from paper_2109_04129_amd import hps  # noqa: E402

pytestmark = pytest.mark.gpu

FREQ = 300e6
ALPHA = 0.5


def _mesh():
    xyz, tri = icosphere(2, 1.0)
    return ellipsoid_mesh(xyz, tri, (1.3, 0.9, 0.6))


def _angles():
    return monostatic_angles([0.0, 37.0, 90.0, 151.0, 180.0], [0.0, 20.0, 45.0, 300.0, 0.0])


def _params(**kw):
    base = dict(freq_hz=FREQ, leaf_max=16, aca_tol=1e-3, terms=2, formulation=1, cfie_alpha=ALPHA)
    base.update(kw)
    return hps.hps_params_default(**base)


def _ctx():
    assert torch.cuda.is_available(), "the GPU tests need a HIP device"
    return hps.hps_create(0, torch.cuda.current_stream().cuda_stream)


def _solve(ctx, N, khat, pol):
    X = torch.zeros((len(khat), N), dtype=torch.complex128, device="cuda")
    st, rcs, ratio = hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
    torch.cuda.synchronize()
    return st, X.cpu().numpy().T.copy(), rcs, ratio


@pytest.fixture(scope="module")
def oracle_cfie():
    xyz, tri = _mesh()
    return xyz, tri, build_hmatrix(xyz, tri, FREQ, 16, 1e-3, workers=8, formulation="cfie", alpha=ALPHA)


@pytest.mark.parametrize("ordering", [0, 1])
def test_cfie_against_oracle(oracle_cfie, ordering):
    xyz, tri, H = oracle_cfie
    khat, pol = _angles()
    print("case: CFIE ellipsoid 480 unknowns, oracle H-matrix, ordering", ordering, flush=True)
    ctx = _ctx()
    try:
        hps.hps_set_mesh(ctx, xyz, tri)
        a = hmatrix_arrays(H)
        hps.hps_set_hmatrix(ctx, _params(ordering=ordering), a["N"], a["perm"], a["group_ptr"], a["near_ts"],
                            a["near_off"], a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        hps.hps_setup(ctx)
        st, X, rcs, ratio = _solve(ctx, H.N, khat, pol)
        B = torch.zeros((len(khat), H.N), dtype=torch.complex128, device="cuda")
        hps.hps_excitation(ctx, khat, pol, B.data_ptr())
        torch.cuda.synchronize()
        Bl = B.cpu().numpy().T
    finally:
        hps.hps_destroy(ctx)
    b = excitation_cfie(H.rwg, FREQ, khat, pol, ALPHA)
    assert np.abs(Bl - b).max() <= 1e-12 * np.abs(b).max()
    order = natural_order(H.M) if ordering == 1 else min_degree_order(group_graph(H))
    x, rt = PowerSeries(H, schur_scaling(H, order)).solve_rwg(b, 2)
    sig = monostatic_rcs(H.rwg, FREQ, khat, pol, x)
    err = per_rhs_rel(X, x).max()
    db = np.abs(10 * np.log10(rcs / sig)).max()
    print("current err %.2e, rcs err %.2e dB, ratio max %.3f" % (err, db, np.max(rt)), flush=True)
    assert err < 1e-10
    assert db < 1e-6
    if ordering == 1:
        assert np.abs(ratio - rt[0]).max() < 1e-9 * np.abs(rt).max()


def _library(params, xyz, tri):
    ctx = _ctx()
    hps.hps_set_mesh(ctx, xyz, tri)
    hps.hps_build_hmatrix(ctx, params)
    return ctx


def test_cfie_library_hmatrix(oracle_cfie):
    """Device-built CFIE H-matrix: its product against the dense oracle
    matrix, and its near blocks against the host-built ones."""
    xyz, tri, H = oracle_cfie
    print("case: CFIE library H-matrix vs dense oracle and host build", flush=True)
    dev = _library(_params(), xyz, tri)
    host = _library(_params(host_near=1), xyz, tri)
    try:
        gd, gh = hps.hps_get_hmatrix(dev), hps.hps_get_hmatrix(host)
        hps.hps_setup(dev)
        assert np.array_equal(gd["near_ts"], gh["near_ts"]) and np.array_equal(gd["perm"], gh["perm"])
        dn = np.abs(gd["near_vals"] - gh["near_vals"]).max() / np.abs(gh["near_vals"]).max()
        N = H.N
        g = torch.Generator().manual_seed(3)
        Xh = torch.complex(torch.randn(4, N, generator=g, dtype=torch.float64),
                           torch.randn(4, N, generator=g, dtype=torch.float64))
        Y = torch.zeros_like(Xh).cuda()
        hps.hps_hmatvec(dev, 4, Xh.cuda().data_ptr(), Y.data_ptr())
        torch.cuda.synchronize()
        Zd = H.op.dense()
        ref = Zd @ Xh.numpy().T
        e = per_rhs_rel(Y.cpu().numpy().T, ref).max()
        print("near dev vs host %.1e, H x vs dense %.1e" % (dn, e), flush=True)
        assert dn < 1e-12
        assert e < 2e-3
    finally:
        hps.hps_destroy(dev)
        hps.hps_destroy(host)


def test_cfie_precision_form(oracle_cfie):
    xyz, tri, _ = oracle_cfie
    khat, pol = _angles()
    print("case: CFIE precision form (FP16 far) vs FP64 four terms", flush=True)
    ref = _library(_params(terms=4), xyz, tri)
    mix = _library(_params(precision=2, refine_passes=1), xyz, tri)
    try:
        hps.hps_setup(ref)
        hps.hps_setup(mix)
        N = hps.hps_num_unknowns(ref)
        _, X4, r4, _ = _solve(ref, N, khat, pol)
        _, Xm, rm, _ = _solve(mix, N, khat, pol)
    finally:
        hps.hps_destroy(ref)
        hps.hps_destroy(mix)
    e = per_rhs_rel(Xm, X4).max()
    db = np.abs(10 * np.log10(rm / r4)).max()
    print("precision form: current %.2e, rcs %.2e dB" % (e, db), flush=True)
    assert e < 1e-3 and db < 0.1


def test_cfie_batch_matches_single():
    xyz1, tri1 = _mesh()
    xyz2, tri2 = icosphere(2, 0.8)
    meshes = [(xyz1, tri1), (xyz2, tri2)]
    khat, pol = _angles()
    R = len(khat)
    print("case: CFIE batch of two vs single contexts", flush=True)
    p = _params()
    b = hps.hps_batch_create(2, 0, torch.cuda.current_stream().cuda_stream)
    singles = []
    try:
        for q, (xyz, tri) in enumerate(meshes):
            hps.hps_batch_set_mesh(b, q, xyz, tri)
        hps.hps_build_hmatrix(b, p)
        hps.hps_setup(b)
        Ns = [hps.hps_problem_unknowns(b, q) for q in range(2)]
        X = torch.zeros(R * sum(Ns), dtype=torch.complex128, device="cuda")
        _, rcs, ratio = hps.hps_solve_planewaves(b, khat, pol, X.data_ptr())
        torch.cuda.synchronize()
        Xb = X.cpu().numpy()
        o = 0
        for q, (xyz, tri) in enumerate(meshes):
            c = _library(p, xyz, tri)
            singles.append(c)
            hps.hps_setup(c)
            _, Xq, rq, tq = _solve(c, Ns[q], khat, pol)
            Xbq = Xb[o:o + Ns[q] * R].reshape(R, Ns[q]).T
            o += Ns[q] * R
            print("problem", q, "diff %.1e" % np.abs(Xbq - Xq).max(), flush=True)
            assert np.abs(Xbq - Xq).max() <= 1e-13 * np.abs(Xq).max()
            assert np.allclose(rcs[q], rq, rtol=1e-12, atol=0)
            assert np.allclose(ratio[q], tq, rtol=1e-12, atol=0)
    finally:
        hps.hps_destroy(b)
        for c in singles:
            hps.hps_destroy(c)


def test_cfie_converged_series_matches_mie():
    """1,920-unknown sphere at ka = 4.19: the CFIE's eq. (45) ratio is well
    below 1, so the adaptive series converges; its backscatter matches Mie
    (the dense CFIE solve of this mesh is 0.04 dB from Mie)."""
    xyz, tri = icosphere(3, 1.0)
    f = 200e6
    khat, pol = np.array([[0.0, 0.0, -1.0]]), np.array([[1.0, 0.0, 0.0]])
    print("case: CFIE sphere 1,920 unknowns, adaptive series vs Mie", flush=True)
    c = _library(hps.hps_params_default(freq_hz=f, leaf_max=64, aca_tol=1e-4, terms=30, series_tol=1e-8,
                                         formulation=1, cfie_alpha=0.5), xyz, tri)
    try:
        hps.hps_setup(c)
        N = hps.hps_num_unknowns(c)
        st, X, rcs, ratio = _solve(c, N, khat, pol)
        stats = hps.hps_stats(c)
    finally:
        hps.hps_destroy(c)
    k = wavenumber(f)
    db = 10 * np.log10(rcs[0] / mie.backscatter_rcs(1.0, k))
    print("ratio %.3f, terms used %s, backscatter vs Mie %.3f dB" % (ratio[0], stats["device"].get("terms_used"), db),
          flush=True)
    assert ratio[0] < 0.5
    assert abs(db) < 0.3


def test_cfie_groups_above_128():
    """CFIE with leaves of up to 300 unknowns: the library cuts groups above
    128 into consecutive pivots, every sub-block of a cut diagonal block kept
    (non-symmetric); currents and RCS do not depend on that blocking."""
    xyz, tri = icosphere(3, 1.0)
    xyz, tri = ellipsoid_mesh(xyz, tri, (1.3, 0.9, 0.6))
    H = build_hmatrix(xyz, tri, FREQ, 300, 1e-3, workers=8, formulation="cfie", alpha=ALPHA)
    sizes = H.groups[:, 1] - H.groups[:, 0]
    print("case: CFIE ellipsoid 1,920 unknowns, leaves <= 300 (max %d)" % sizes.max(), flush=True)
    assert sizes.max() > 128
    khat, pol = _angles()
    ctx = _ctx()
    try:
        hps.hps_set_mesh(ctx, xyz, tri)
        a = hmatrix_arrays(H)
        hps.hps_set_hmatrix(ctx, _params(leaf_max=300), a["N"], a["perm"], a["group_ptr"], a["near_ts"],
                            a["near_off"], a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        hps.hps_setup(ctx)
        assert hps.hps_stats(ctx)["device"]["groups"] > H.M
        st, X, rcs, ratio = _solve(ctx, H.N, khat, pol)
    finally:
        hps.hps_destroy(ctx)
    b = excitation_cfie(H.rwg, FREQ, khat, pol, ALPHA)
    x, _ = PowerSeries(H, schur_scaling(H, min_degree_order(group_graph(H)))).solve_rwg(b, 2)
    sig = monostatic_rcs(H.rwg, FREQ, khat, pol, x)
    err = per_rhs_rel(X, x).max()
    print("current err %.2e" % err, flush=True)
    assert err < 1e-10
    assert np.abs(10 * np.log10(rcs / sig)).max() < 1e-6


def test_cfie_arbitrary_rhs_and_graph_replay(oracle_cfie):
    """hps_solve_rhs on random right-hand sides against the oracle series
    (left and right coefficients), and repeated graph replays of that solve
    against eager launches, bit for bit."""
    xyz, tri, H = oracle_cfie
    R = 19
    print("case: CFIE arbitrary RHS (R=19), graph replays vs eager", flush=True)
    g = torch.Generator().manual_seed(11)
    Bh = torch.complex(torch.randn(R, H.N, generator=g, dtype=torch.float64),
                       torch.randn(R, H.N, generator=g, dtype=torch.float64))
    a = hmatrix_arrays(H)
    outs = {}
    for graphs in (0, 1):
        ctx = _ctx()
        try:
            hps.hps_set_mesh(ctx, xyz, tri)
            hps.hps_set_hmatrix(ctx, _params(graphs=graphs), a["N"], a["perm"], a["group_ptr"], a["near_ts"],
                                a["near_off"], a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"],
                                a["far_uv"])
            hps.hps_setup(ctx)
            B = Bh.cuda()
            outs[graphs] = []
            for _ in range(3):
                X = torch.zeros_like(B)
                hps.hps_solve_rhs(ctx, R, B.data_ptr(), X.data_ptr())
                torch.cuda.synchronize()
                outs[graphs].append(X.cpu().numpy().T.copy())
        finally:
            hps.hps_destroy(ctx)
    for o in outs[0][1:] + outs[1]:
        assert np.array_equal(o, outs[0][0])
    x, _ = PowerSeries(H, schur_scaling(H, min_degree_order(group_graph(H)))).solve_rwg(Bh.numpy().T, 2)
    err = per_rhs_rel(outs[1][0], x).max()
    print("current err %.2e" % err, flush=True)
    assert err < 1e-10


def test_cfie_tile_shapes_bitwise(oracle_cfie, tmp_path):
    """The non-symmetric setup on the pipelined shapes (packed Schur tiles of
    upper and lower blocks) and on the plain-register 32 x 64 tile gives
    bitwise the currents of the 32 x 32 tile; packing uses fewer 16-column
    block slots for the same blocks."""
    import json
    xyz, tri, H = oracle_cfie
    khat, pol = _angles()
    print("case: CFIE ellipsoid 480 unknowns, tile shapes 0, 7, 11, 12", flush=True)
    a = hmatrix_arrays(H)
    out, split = {}, {}
    for shape in (0, 7, 11, 12):
        path = tmp_path / ("shape%d.json" % shape)
        path.write_text(json.dumps({"entries": [{"class": c, "shape": shape}
                                                for c in ("sweep", "dinv", "far1", "far2", "near", "schur")]}))
        ctx = _ctx()
        try:
            hps.hps_set_tuning(ctx, str(path))
            hps.hps_set_mesh(ctx, xyz, tri)
            hps.hps_set_hmatrix(ctx, _params(), a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"],
                                a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
            hps.hps_setup(ctx)
            out[shape] = _solve(ctx, H.N, khat, pol)
            dev = hps.hps_stats(ctx)["device"]
            assert dev["tuning"]["shapes"]["schur"] == shape
            split[shape] = dev["schedule_split"]
        finally:
            hps.hps_destroy(ctx)
    for shape in (7, 11, 12):
        assert np.array_equal(out[shape][1], out[0][1]), "shape %d" % shape
        assert np.array_equal(out[shape][2], out[0][2]), "shape %d" % shape
    s7, s12 = split[7], split[12]
    print("column-block slots: shape 7 %d of %d used, shape 12 %d of %d used" % (
        s7["schur_col_active"], s7["schur_col_slots"], s12["schur_col_active"], s12["schur_col_slots"]), flush=True)
    assert s12["schur_col_active"] == s7["schur_col_active"] > 0
    assert s12["schur_col_slots"] < s7["schur_col_slots"]
