"""Tile shapes of the grouped complex GEMM (the autotuner's choices, shape 5
the LDS-staged kernel, 11 and 12 the pipelined ones): every
shape sums the same products in the same order for each output element, so
setup and solve results are bitwise those of the 32 x 32 shape.  Checked on
the oracle's H-matrix of the 1,920-unknown sphere with 37 RHS (two column
tiles of 32, one of them ragged; one ragged 64- and 128-column tile), FP64
and the FP32 precision form, with every class (Schur updates, sweeps, D^-1,
far stages, near product) forced to each shape; the FP64 result is also held
against the oracle's two-term series (1e-10)."""

import json

import numpy as np
import pytest

from oracle.planewave import excitation
from oracle.scaling import group_graph, min_degree_order, schur_scaling
from oracle.series import PowerSeries
from workloads import monostatic_angles
from hmat_io import hmatrix_arrays, per_rhs_rel

torch = pytest.importorskip("torch")
from paper_2109_04129_amd import hps  # noqa: E402

pytestmark = pytest.mark.gpu

CLASSES = ["sweep", "dinv", "far1", "far2", "near", "schur"]


def _run(w, H, shape, precision, tmp_path, nrhs=37, stats=None):
    path = tmp_path / ("shape%d.json" % shape)
    path.write_text(json.dumps({"entries": [{"class": c, "shape": shape} for c in CLASSES]}))
    ctx = hps.hps_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        hps.hps_set_tuning(ctx, str(path))
        hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
        p = hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"], aca_tol=1e-3, terms=2,
                                   precision=precision, refine_passes=1 if precision else 0)
        a = hmatrix_arrays(H)
        hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"], a["near_vals"],
                            a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        hps.hps_setup(ctx)
        th = np.linspace(0.0, 180.0, 37)[:nrhs]
        khat, pol = monostatic_angles(th, np.zeros_like(th))
        X = torch.zeros((nrhs, H.N), dtype=torch.complex128, device="cuda")
        st, rcs, ratio = hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
        Y = torch.zeros_like(X)
        hps.hps_hmatvec(ctx, nrhs, X.data_ptr(), Y.data_ptr())
        torch.cuda.synchronize()
        dev = hps.hps_stats(ctx)["device"]
        if stats is not None:
            stats.append(dev)
        used = dev["tuning"]["shapes"]
        # the setup's Schur updates have no one-column launches: shape 6 means 0 there
        assert all(v == (0 if (c == "schur" and shape == 6) else shape) for c, v in used.items()), used
        return X.cpu().numpy(), Y.cpu().numpy(), rcs, ratio, khat, pol
    finally:
        hps.hps_destroy(ctx)


@pytest.mark.parametrize("precision", [0, 2])
def test_tile_shapes_bitwise(c0_workload, c0_hmatrix, precision, tmp_path):
    w, H = c0_workload, c0_hmatrix
    print("case: tile shapes 0-12, sphere 1,920 unknowns, 37 RHS, precision %d" % precision, flush=True)
    X0, Y0, rcs0, ratio0, khat, pol = _run(w, H, 0, precision, tmp_path)
    for shape in range(1, 13):          # 6 (the one-column kernel) falls back to 0 for 37 columns
        X, Y, rcs, ratio, _, _ = _run(w, H, shape, precision, tmp_path)
        assert np.array_equal(X, X0), "shape %d: currents differ (max %.3e)" % (shape, np.max(np.abs(X - X0)))
        assert np.array_equal(Y, Y0), "shape %d: H x differs" % shape
        assert np.array_equal(rcs, rcs0) and np.array_equal(ratio, ratio0), "shape %d" % shape
    if precision == 0:
        b = excitation(H.rwg, w["freq_hz"], khat, pol)
        x_ref, _ = PowerSeries(H, schur_scaling(H, min_degree_order(group_graph(H)))).solve_rwg(b, 2)
        err = per_rhs_rel(X0.T, x_ref).max()
        print("shape 0 vs oracle: %.2e" % err, flush=True)
        assert err < 1e-10


def test_packed_schur_tiles(c0_workload, c0_hmatrix, tmp_path):
    """The pipelined shape deals the 16-column blocks of single-term Schur
    targets four to a tile: the same blocks in fewer tile slots than the
    unpacked 32 x 64 tile of shape 7, and bitwise the same results."""
    w, H = c0_workload, c0_hmatrix
    print("case: packed Schur tiles, shape 12 vs 7, sphere 1,920 unknowns", flush=True)
    s7, s12 = [], []
    X7, Y7, rcs7, _, _, _ = _run(w, H, 7, 0, tmp_path, stats=s7)
    X12, Y12, rcs12, _, _, _ = _run(w, H, 12, 0, tmp_path, stats=s12)
    a7, a12 = s7[0]["schedule_split"], s12[0]["schedule_split"]
    print("column-block slots: shape 7 %d of %d used, shape 12 %d of %d used" % (
        a7["schur_col_active"], a7["schur_col_slots"], a12["schur_col_active"], a12["schur_col_slots"]), flush=True)
    assert a12["schur_col_active"] == a7["schur_col_active"] > 0
    assert a12["schur_col_slots"] < a7["schur_col_slots"]
    assert np.array_equal(X12, X7) and np.array_equal(Y12, Y7) and np.array_equal(rcs12, rcs7)


def test_one_column_vector_kernel(c0_workload, c0_hmatrix, tmp_path):
    """Shape 6 (the vector-ALU matrix-vector kernel for one-column FP64
    solves) sums in another order: its one-RHS currents, RCS, ratio and H x
    agree with the MFMA kernel's to rounding (1e-13) and with the oracle's
    two-term series (1e-10)."""
    w, H = c0_workload, c0_hmatrix
    print("case: one-column solve, vector kernel vs 32 x 32 MFMA tiles, 1,920 unknowns", flush=True)
    X0, Y0, rcs0, ratio0, khat, pol = _run(w, H, 0, 0, tmp_path, nrhs=1)
    X6, Y6, rcs6, ratio6, _, _ = _run(w, H, 6, 0, tmp_path, nrhs=1)
    e_x = np.linalg.norm(X6 - X0) / np.linalg.norm(X0)
    e_y = np.linalg.norm(Y6 - Y0) / np.linalg.norm(Y0)
    print("vector vs MFMA: currents %.2e, H x %.2e" % (e_x, e_y), flush=True)
    assert e_x < 1e-13 and e_y < 1e-13
    assert abs(rcs6[0] / rcs0[0] - 1) < 1e-12 and abs(ratio6[0] / ratio0[0] - 1) < 1e-12
    b = excitation(H.rwg, w["freq_hz"], khat, pol)
    x_ref, _ = PowerSeries(H, schur_scaling(H, min_degree_order(group_graph(H)))).solve_rwg(b, 2)
    assert per_rhs_rel(X6.T, x_ref).max() < 1e-10


@pytest.mark.parametrize("kpull", [64, 10 ** 9])
def test_pull_sweeps(c0_workload, c0_hmatrix, kpull, tmp_path):
    """Sweep targets whose contraction is at most sweep_pull_kmax take all
    their terms in one tile set (pull) instead of one per source level
    (push): the sums run in another order, so currents, RCS, ratios and the
    H-matrix product agree with the push form to rounding (1e-12) and with
    the oracle's two-term series (1e-10).  kpull = 64 mixes both forms in one
    launch; 10^9 pulls every target."""
    w, H = c0_workload, c0_hmatrix
    print("case: pull sweeps (kmax %d) vs push, sphere 1,920 unknowns, 37 RHS" % kpull, flush=True)
    X0, Y0, rcs0, ratio0, khat, pol = _run(w, H, 0, 0, tmp_path)
    path = tmp_path / "pull.json"
    path.write_text(json.dumps({"sweep_pull_kmax": kpull, "entries": []}))
    ctx = hps.hps_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        hps.hps_set_tuning(ctx, str(path))
        hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
        p = hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"], aca_tol=1e-3, terms=2)
        a = hmatrix_arrays(H)
        hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"], a["near_vals"],
                            a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        hps.hps_setup(ctx)
        X = torch.zeros((len(khat), H.N), dtype=torch.complex128, device="cuda")
        _, rcs, ratio = hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
        torch.cuda.synchronize()
        assert hps.hps_stats(ctx)["device"]["tuning"]["sweep_pull_kmax"] == kpull
        X = X.cpu().numpy()
    finally:
        hps.hps_destroy(ctx)
    e_push = per_rhs_rel(X.T, X0.T).max()
    b = excitation(H.rwg, w["freq_hz"], khat, pol)
    x_ref, _ = PowerSeries(H, schur_scaling(H, min_degree_order(group_graph(H)))).solve_rwg(b, 2)
    e_or = per_rhs_rel(X.T, x_ref).max()
    print("pull vs push %.2e, vs oracle %.2e" % (e_push, e_or), flush=True)
    assert e_push < 1e-12 and e_or < 1e-10
    assert np.max(np.abs(rcs / rcs0 - 1)) < 1e-10 and np.max(np.abs(ratio / ratio0 - 1)) < 1e-10
