"""CPU checks of the C ABI: the library loads, exports every function that
include/hps.h declares, validates its inputs, and its host-side H-matrix
build (tree, near/far split, EFIE entries, ACA) agrees with the oracle.
No device work is launched here."""

import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2109_04129_amd import hps
from workloads import icosphere
from conftest import ROOT, rel

HEADER = os.path.join(ROOT, "include", "hps.h")


def test_exports_match_header():
    decl = set(re.findall(r"\b(hps_[a-z_]+)\s*\(", open(HEADER).read()))
    out = subprocess.run(["nm", "-D", "--defined-only", hps.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(hps_[a-z_]+)\b", out))
    assert decl, "no declarations parsed"
    assert decl <= exported, decl - exported
    assert set(hps.EXPORTS) == decl
    L = hps.lib()
    for name in decl:
        assert hasattr(L, name)


def test_host_context_and_errors():
    ctx = hps.hps_create(-1)
    try:
        with pytest.raises(hps.HpsError) as e:
            hps.hps_setup(ctx)
        assert e.value.status == -5                     # ESTATE: no H-matrix yet
        xyz, tri = icosphere(1)
        with pytest.raises(hps.HpsError) as e:
            hps.hps_set_mesh(ctx, xyz, tri[1:])         # open mesh
        assert e.value.status == -1
        bad = tri.copy()
        bad[0] = bad[0][[0, 2, 1]]
        with pytest.raises(hps.HpsError):
            hps.hps_set_mesh(ctx, xyz, bad)             # inconsistent orientation
        hps.hps_set_mesh(ctx, xyz, tri)
        assert hps.hps_num_unknowns(ctx) == 120
        p = hps.hps_params_default(freq_hz=0.0)
        with pytest.raises(hps.HpsError):
            hps.hps_build_hmatrix(ctx, p)               # freq must be > 0
        for bad in (-1, 3):                             # graphs: 0, 1 or 2
            with pytest.raises(hps.HpsError) as e:
                hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=300e6, leaf_max=16, graphs=bad))
            assert e.value.status == -1
        p = hps.hps_params_default(freq_hz=300e6, leaf_max=16, graphs=2)
        hps.hps_build_hmatrix(ctx, p)
        with pytest.raises(hps.HpsError) as e:
            hps.hps_setup(ctx)                          # host-only context
        assert e.value.status == -3
    finally:
        hps.hps_destroy(ctx)


def test_host_hmatrix_matches_oracle(c0_workload, c0_hmatrix, c0_dense):
    w, H = c0_workload, c0_hmatrix
    ctx = hps.hps_create(-1)
    try:
        hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
        hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"],
                                                          aca_tol=w["aca_tol"]))
        L = hps.hps_get_hmatrix(ctx)
    finally:
        hps.hps_destroy(ctx)
    # integer structure: bit-exact
    assert np.array_equal(L["perm"], H.perm)
    assert np.array_equal(L["group_ptr"], np.r_[H.groups[:, 0], H.N])
    keys = [tuple(x) for x in L["near_ts"].reshape(-1, 2)]
    assert keys == sorted(H.near)
    assert np.array_equal(L["far_rng"].reshape(-1, 4), np.array([f[:4] for f in H.far]))
    # near entries: same quadrature definition, different code -> rounding only
    for b, k in enumerate(keys):
        blk = L["near_vals"][L["near_off"][b]:L["near_off"][b + 1]].reshape(H.near[k].shape)
        assert np.abs(blk - H.near[k]).max() <= 1e-13 * np.abs(H.near[k]).max()
    # far blocks: the library's own ACA within 2 eps of the dense matrix overall
    P = H.perm
    Zt = c0_dense[np.ix_(P, P)]
    Zh = H.dense_near()
    for b, (tlo, thi, slo, shi) in enumerate(L["far_rng"].reshape(-1, 4)):
        r, m, n = L["far_rank"][b], thi - tlo, shi - slo
        uv = L["far_uv"][L["far_off"][b]:L["far_off"][b + 1]]
        B = uv[:m * r].reshape(r, m).T @ uv[m * r:].reshape(r, n)
        Zh[tlo:thi, slo:shi] = B
        Zh[slo:shi, tlo:thi] = B.T
    assert rel(Zh, Zt) <= 2e-3


def _batch_meshes():
    from workloads import ellipsoid_mesh
    xyz1, tri1 = icosphere(1, 1.0)
    xyz2, tri2 = icosphere(2, 1.0)
    xyz3, tri3 = ellipsoid_mesh(xyz2, tri2, (1.3, 0.9, 0.6))
    return [(xyz1, tri1), (xyz3, tri3), (0.8 * xyz2, tri2)]


def test_host_batch_merge_and_errors():
    """A batch context merges its problems into one block-diagonal H-matrix
    whose blocks are exactly those of single-problem contexts, shifted by the
    offsets of the problems before them; misuse is rejected."""
    meshes = _batch_meshes()
    p = hps.hps_params_default(freq_hz=300e6, leaf_max=16)
    with pytest.raises(hps.HpsError) as e:
        hps.hps_batch_create(0, -1)
    assert e.value.status == -1
    ctx = hps.hps_batch_create(len(meshes), -1)
    single = []
    try:
        assert hps.hps_num_problems(ctx) == 3
        xyz, tri = meshes[0]
        with pytest.raises(hps.HpsError) as e:
            hps.hps_set_mesh(ctx, xyz, tri)                 # batch takes hps_batch_set_mesh
        assert e.value.status == -1
        with pytest.raises(hps.HpsError) as e:
            hps.hps_batch_set_mesh(ctx, 3, xyz, tri)        # problem index out of range
        assert e.value.status == -1
        hps.hps_batch_set_mesh(ctx, 0, xyz, tri)
        with pytest.raises(hps.HpsError) as e:
            hps.hps_build_hmatrix(ctx, p)                   # meshes 1 and 2 missing
        assert e.value.status == -5
        for q in (1, 2):
            hps.hps_batch_set_mesh(ctx, q, *meshes[q])
        Ns = [hps.hps_problem_unknowns(ctx, q) for q in range(3)]
        assert Ns == [120, 480, 480]
        assert hps.hps_num_unknowns(ctx) == sum(Ns)
        hps.hps_build_hmatrix(ctx, p)
        B = hps.hps_get_hmatrix(ctx)
        with pytest.raises(hps.HpsError) as e:
            hps.hps_setup(ctx)                              # host-only context
        assert e.value.status == -3
        for q in range(3):
            c = hps.hps_create(-1)
            single.append(c)
            hps.hps_set_mesh(c, *meshes[q])
            hps.hps_build_hmatrix(c, p)
            with pytest.raises(hps.HpsError) as e:
                hps.hps_batch_set_mesh(c, 0, *meshes[q])    # not a batch context
            assert e.value.status == -1
        S = [hps.hps_get_hmatrix(c) for c in single]
        noff = np.concatenate([[0], np.cumsum(Ns)])
        goff = np.concatenate([[0], np.cumsum([len(s["group_ptr"]) - 1 for s in S])])
        assert np.array_equal(B["perm"], np.concatenate([s["perm"] + o for s, o in zip(S, noff)]))
        assert np.array_equal(B["group_ptr"], np.concatenate(
            [[0]] + [s["group_ptr"][1:] + o for s, o in zip(S, noff)]))
        assert np.array_equal(B["near_ts"], np.concatenate([s["near_ts"] + g for s, g in zip(S, goff)]))
        assert np.array_equal(B["near_vals"], np.concatenate([s["near_vals"] for s in S]))
        assert np.array_equal(B["far_rng"], np.concatenate([s["far_rng"] + o for s, o in zip(S, noff)]))
        assert np.array_equal(B["far_rank"], np.concatenate([s["far_rank"] for s in S]))
        assert np.array_equal(B["far_uv"], np.concatenate([s["far_uv"] for s in S]))
        # no far block and no near block couples two problems
        rng = B["far_rng"].reshape(-1, 4) - np.array([0, 1, 0, 1])     # inclusive ends
        prob = np.searchsorted(noff, rng, side="right") - 1
        assert np.all(prob == prob[:, :1])
        ts = B["near_ts"].reshape(-1, 2)
        gp = np.searchsorted(goff, ts, side="right") - 1
        assert np.all(gp[:, 0] == gp[:, 1])
        # per-problem installs must share one parameter set
        p2 = hps.hps_params_default(freq_hz=310e6, leaf_max=16)
        s0 = S[0]
        hps.hps_batch_set_hmatrix(ctx, 0, p, Ns[0], s0["perm"], s0["group_ptr"], s0["near_ts"], s0["near_off"],
                                  s0["near_vals"], s0["far_rng"], s0["far_rank"], s0["far_off"], s0["far_uv"])
        with pytest.raises(hps.HpsError) as e:
            hps.hps_batch_set_hmatrix(ctx, 0, p2, Ns[0], s0["perm"], s0["group_ptr"], s0["near_ts"],
                                      s0["near_off"], s0["near_vals"], s0["far_rng"], s0["far_rank"],
                                      s0["far_off"], s0["far_uv"])
        assert e.value.status == -1
    finally:
        hps.hps_destroy(ctx)
        for c in single:
            hps.hps_destroy(c)



def test_groups_above_128_are_cut(c0_workload):
    """Leaves of up to 256 unknowns: the library holds groups of at most 128,
    and its near field is the oracle's (groups of up to 256) entry for entry."""
    from oracle.hmatrix import build_hmatrix
    from hmat_io import dense_near_from_arrays
    w = c0_workload
    H = build_hmatrix(w["xyz"], w["tri"], w["freq_hz"], 256, w["aca_tol"], workers=min(8, os.cpu_count() or 1))
    assert (H.groups[:, 1] - H.groups[:, 0]).max() > 128
    ctx = hps.hps_create(-1)
    try:
        hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
        hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=256, aca_tol=w["aca_tol"]))
        L = hps.hps_get_hmatrix(ctx)
        L["N"] = hps.hps_num_unknowns(ctx)
        # installing the oracle's H-matrix cuts its groups the same way
        from hmat_io import hmatrix_arrays
        a = hmatrix_arrays(H)
        hps.hps_set_hmatrix(ctx, hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=256), a["N"], a["perm"],
                            a["group_ptr"], a["near_ts"], a["near_off"], a["near_vals"], a["far_rng"],
                            a["far_rank"], a["far_off"], a["far_uv"])
        I = hps.hps_get_hmatrix(ctx)
    finally:
        hps.hps_destroy(ctx)
    for X in (L, I):
        sizes = np.diff(X["group_ptr"])
        assert sizes.max() <= 128 and sizes.min() >= 1
        assert np.array_equal(X["perm"], H.perm)
    assert np.array_equal(I["group_ptr"], L["group_ptr"])
    Zo = H.dense_near()
    assert np.array_equal(dense_near_from_arrays(I), Zo)          # pure re-layout of the same values
    assert np.abs(dense_near_from_arrays(L) - Zo).max() <= 1e-13 * np.abs(Zo).max()
    assert np.array_equal(L["far_rng"], I["far_rng"])


def test_minimum_box_side_matches_oracle(c0_workload):
    """Leaves of at least half a wavelength (0.75 m at 200 MHz): the library's
    tree and near/far split equal the oracle's (groups above 128 unknowns cut
    into consecutive pivots), and its near field equals the oracle's."""
    from oracle.hmatrix import build_hmatrix
    from hmat_io import dense_near_from_arrays
    w = c0_workload
    box = 0.5 * 299792458.0 / w["freq_hz"]
    H = build_hmatrix(w["xyz"], w["tri"], w["freq_hz"], 64, w["aca_tol"], workers=min(8, os.cpu_count() or 1),
                      box_min=box)
    assert (H.groups[:, 1] - H.groups[:, 0]).max() > 64
    ctx = hps.hps_create(-1)
    try:
        hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
        hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=64, aca_tol=w["aca_tol"],
                                                          leaf_box_min=box))
        L = hps.hps_get_hmatrix(ctx)
    finally:
        hps.hps_destroy(ctx)
    assert np.array_equal(L["perm"], H.perm)
    assert set(H.groups[:, 0]) <= set(L["group_ptr"][:-1])          # library groups refine the oracle's
    assert np.diff(L["group_ptr"]).max() <= 128
    assert np.array_equal(L["far_rng"].reshape(-1, 4), np.array([f[:4] for f in H.far]).reshape(-1, 4))
    Zo = H.dense_near()
    assert np.abs(dense_near_from_arrays(L) - Zo).max() <= 1e-13 * np.abs(Zo).max()


def test_open_plate_matches_oracle():
    """Open sheet: hps_set_mesh rejects the rim, hps_set_open_mesh takes it;
    the library's RWG numbering, tree, near/far split and near entries equal
    the oracle's (open_surface=True)."""
    from oracle.hmatrix import build_hmatrix
    from workloads import workload
    w = workload("plate_2lambda_300MHz")
    H = build_hmatrix(w["xyz"], w["tri"], w["freq_hz"], w["leaf_max"], w["aca_tol"],
                      workers=min(8, os.cpu_count() or 1), open_surface=True)
    ctx = hps.hps_create(-1)
    try:
        with pytest.raises(hps.HpsError) as e:
            hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
        assert e.value.status == -1
        hps.hps_set_open_mesh(ctx, w["xyz"], w["tri"])
        assert hps.hps_num_unknowns(ctx) == H.N == 1160
        hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"],
                                                          aca_tol=w["aca_tol"]))
        L = hps.hps_get_hmatrix(ctx)
    finally:
        hps.hps_destroy(ctx)
    assert np.array_equal(L["perm"], H.perm)
    assert np.array_equal(L["group_ptr"], np.r_[H.groups[:, 0], H.N])
    assert np.array_equal(L["far_rng"].reshape(-1, 4), np.array([f[:4] for f in H.far]))
    keys = [tuple(x) for x in L["near_ts"].reshape(-1, 2)]
    assert keys == sorted(H.near)
    for b, k in enumerate(keys):
        blk = L["near_vals"][L["near_off"][b]:L["near_off"][b + 1]].reshape(H.near[k].shape)
        assert np.abs(blk - H.near[k]).max() <= 1e-13 * np.abs(H.near[k]).max()


# ---------------------------------------------------------------- CFIE (eq. 8)
def test_cfie_parameters_checked():
    from workloads import icosphere, workload
    xyz, tri = icosphere(1, 1.0)
    h = hps.hps_create(-1, None)
    try:
        hps.hps_set_mesh(h, xyz, tri)
        for bad in (dict(formulation=2), dict(formulation=1, cfie_alpha=1.5), dict(formulation=1, cfie_alpha=-0.1)):
            with pytest.raises(hps.HpsError) as e:
                hps.hps_build_hmatrix(h, hps.hps_params_default(freq_hz=300e6, leaf_max=16, **bad))
            assert e.value.status == -1
    finally:
        hps.hps_destroy(h)
    w = workload("plate_2lambda_300MHz")
    h = hps.hps_create(-1, None)
    try:
        hps.hps_set_open_mesh(h, w["xyz"], w["tri"])
        with pytest.raises(hps.HpsError) as e:
            hps.hps_build_hmatrix(h, hps.hps_params_default(freq_hz=300e6, leaf_max=16, formulation=1))
        assert e.value.status == -1 and "closed" in str(e.value)
    finally:
        hps.hps_destroy(h)


def test_cfie_host_build_matches_oracle_entries():
    """Host-built CFIE H-matrix: every ordered near pair is present, the near
    blocks equal the oracle's CFIE entries to rounding, and the far blocks
    approximate the dense oracle matrix to the ACA tolerance."""
    from oracle.mfie import CFIEOperator
    from oracle.rwg import build_rwg
    from workloads import ellipsoid_mesh, icosphere
    xyz, tri = icosphere(2, 1.0)
    xyz, tri = ellipsoid_mesh(xyz, tri, (1.3, 0.9, 0.6))
    h = hps.hps_create(-1, None)
    try:
        hps.hps_set_mesh(h, xyz, tri)
        hps.hps_build_hmatrix(h, hps.hps_params_default(freq_hz=300e6, leaf_max=16, aca_tol=1e-3, formulation=1,
                                                        cfie_alpha=0.5))
        g = hps.hps_get_hmatrix(h)
    finally:
        hps.hps_destroy(h)
    Z = CFIEOperator(build_rwg(xyz, tri), 300e6, 0.5).dense()
    perm, gp, ts = g["perm"], g["group_ptr"], g["near_ts"].reshape(-1, 2)
    pairs = set(map(tuple, ts))
    assert all((s, t) in pairs for t, s in pairs)
    assert np.any(ts[:, 0] > ts[:, 1])
    worst = 0.0
    for b, (t, s) in enumerate(ts):
        B = g["near_vals"][g["near_off"][b]:g["near_off"][b + 1]].reshape(gp[t + 1] - gp[t], gp[s + 1] - gp[s])
        ref = Z[np.ix_(perm[gp[t]:gp[t + 1]], perm[gp[s]:gp[s + 1]])]
        worst = max(worst, np.abs(B - ref).max() / np.abs(ref).max())
    assert worst < 1e-12
    fr = g["far_rng"].reshape(-1, 4)
    num = den = 0.0
    for b, (a0, a1, b0, b1) in enumerate(fr):
        r, o = g["far_rank"][b], g["far_off"][b]
        U = g["far_uv"][o:o + (a1 - a0) * r].reshape(r, a1 - a0).T
        V = g["far_uv"][o + (a1 - a0) * r:o + (a1 - a0 + b1 - b0) * r].reshape(r, b1 - b0).T
        ref = Z[np.ix_(perm[a0:a1], perm[b0:b1])]
        num += np.linalg.norm(U @ V.T - ref) ** 2
        den += np.linalg.norm(ref) ** 2
    assert math.sqrt(num / den) < 2e-3


# ---------------------------------------------------------------- RWG table and H-matrix files
def test_rwg_table_matches_oracle():
    """hps_rwg: the library's RWG functions (edge vertices, T+ / T-, free
    vertices) equal the oracle's, for a closed sphere, an open plate and a
    batch of two meshes (ids counted in the concatenated meshes)."""
    from oracle.rwg import build_rwg
    from workloads import workload
    xyz, tri = icosphere(2)
    w = workload("plate_2lambda_300MHz")
    cases = [(xyz, tri, False), (w["xyz"], w["tri"], True)]
    for x, t, open_ in cases:
        o = build_rwg(x, t, allow_open=open_)
        ctx = hps.hps_create(-1)
        try:
            with pytest.raises(hps.HpsError) as e:
                hps.hps_rwg(ctx)
            assert e.value.status == -5                 # ESTATE: no mesh yet
            (hps.hps_set_open_mesh if open_ else hps.hps_set_mesh)(ctx, x, t)
            ev, tpm, fv = hps.hps_rwg(ctx)
        finally:
            hps.hps_destroy(ctx)
        assert np.array_equal(ev, o["edges"])
        assert np.array_equal(tpm, np.stack([o["tplus"], o["tminus"]], 1))
        assert np.array_equal(fv, np.stack([o["vplus"], o["vminus"]], 1))
    x2, t2 = icosphere(1, 0.5)
    b = hps.hps_batch_create(2, -1)
    try:
        hps.hps_batch_set_mesh(b, 0, xyz, tri)
        hps.hps_batch_set_mesh(b, 1, x2, t2)
        ev, tpm, fv = hps.hps_rwg(b)
    finally:
        hps.hps_destroy(b)
    o0, o1 = build_rwg(xyz, tri), build_rwg(x2, t2)
    assert np.array_equal(ev, np.r_[o0["edges"], o1["edges"] + len(xyz)])
    assert np.array_equal(tpm[:, 0], np.r_[o0["tplus"], o1["tplus"] + len(tri)])
    assert np.array_equal(fv[:, 1], np.r_[o0["vminus"], o1["vminus"] + len(xyz)])


@pytest.mark.parametrize("formulation", [0, 1])
def test_hmatrix_file_round_trip(tmp_path, formulation):
    """hps_export_hmatrix / hps_import_hmatrix: the imported H-matrix equals
    the exported one bit for bit (EFIE and CFIE layouts); missing, foreign
    and truncated files give HPS_EIO, a file for another mesh HPS_EINVAL, and
    a failed import leaves the installed H-matrix in place."""
    xyz, tri = icosphere(2)
    p = hps.hps_params_default(freq_hz=300e6, leaf_max=16, formulation=formulation, cfie_alpha=0.3)
    path = str(tmp_path / "h.bin")
    a = hps.hps_create(-1)
    try:
        with pytest.raises(hps.HpsError) as e:
            hps.hps_export_hmatrix(a, path)
        assert e.value.status == -5                     # nothing to export yet
        hps.hps_set_mesh(a, xyz, tri)
        hps.hps_build_hmatrix(a, p)
        hps.hps_export_hmatrix(a, path)
        ref = hps.hps_get_hmatrix(a)
    finally:
        hps.hps_destroy(a)
    b = hps.hps_create(-1)
    try:
        with pytest.raises(hps.HpsError) as e:
            hps.hps_import_hmatrix(b, path)
        assert e.value.status == -5                     # mesh first
        hps.hps_set_mesh(b, xyz, tri)
        hps.hps_import_hmatrix(b, path)
        got = hps.hps_get_hmatrix(b)
        for k in ref:
            assert ref[k].dtype == got[k].dtype and np.array_equal(ref[k], got[k]), k
        data = open(path, "rb").read()
        bad = [(str(tmp_path / "missing.bin"), None), (str(tmp_path / "foreign.bin"), b"NOTHMAT1" + data[8:]),
               (str(tmp_path / "short.bin"), data[:-16]), (str(tmp_path / "long.bin"), data + b"\0" * 8)]
        for name, content in bad:
            if content is not None:
                open(name, "wb").write(content)
            with pytest.raises(hps.HpsError) as e:
                hps.hps_import_hmatrix(b, name)
            assert e.value.status == -6, name
        assert np.array_equal(hps.hps_get_hmatrix(b)["near_vals"], ref["near_vals"])
    finally:
        hps.hps_destroy(b)
    c = hps.hps_create(-1)
    try:
        x3, t3 = icosphere(1)
        hps.hps_set_mesh(c, x3, t3)
        with pytest.raises(hps.HpsError) as e:
            hps.hps_import_hmatrix(c, path)
        assert e.value.status == -1                     # another mesh
    finally:
        hps.hps_destroy(c)
    bt = hps.hps_batch_create(1, -1)
    try:
        hps.hps_batch_set_mesh(bt, 0, xyz, tri)
        with pytest.raises(hps.HpsError) as e:
            hps.hps_import_hmatrix(bt, path)
        assert e.value.status == -1                     # batch context
    finally:
        hps.hps_destroy(bt)


@pytest.mark.parametrize("eta", [0.0, 1.0])
def test_eta_partition_matches_oracle(eta):
    """hps_params.eta (eq. 10): below sqrt(3) the library's near / far split
    of the 480-unknown sphere equals the oracle's (more near blocks than the
    touch test; eta = 0 leaves no far block), and its near field equals the
    oracle's entries."""
    from oracle.hmatrix import build_hmatrix
    from hmat_io import dense_near_from_arrays
    xyz, tri = icosphere(2, 1.0)
    H = build_hmatrix(xyz, tri, 300e6, 16, 1e-3, workers=min(8, os.cpu_count() or 1), eta=eta)
    ctx = hps.hps_create(-1)
    try:
        hps.hps_set_mesh(ctx, xyz, tri)
        with pytest.raises(hps.HpsError) as e:
            hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=300e6, leaf_max=16, eta=-1.0))
        assert e.value.status == -1
        hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=300e6, leaf_max=16, aca_tol=1e-3, eta=eta))
        L = hps.hps_get_hmatrix(ctx)
    finally:
        hps.hps_destroy(ctx)
    assert np.array_equal(L["perm"], H.perm)
    assert [tuple(x) for x in L["near_ts"].reshape(-1, 2)] == sorted(H.near)
    assert np.array_equal(L["far_rng"].reshape(-1, 4), np.array([f[:4] for f in H.far], dtype=np.int64).reshape(-1, 4))
    if eta == 0.0:
        assert len(H.far) == 0
    Zo = H.dense_near()
    assert np.abs(dense_near_from_arrays(L) - Zo).max() <= 1e-13 * np.abs(Zo).max()


def test_device_mem_cap_enomem_before_device():
    """device_mem_cap: hps_setup plans on the host and returns HPS_ENOMEM
    before touching a device when the plan's device memory exceeds the cap
    (here on a host-only context, which would otherwise fail with
    HPS_EDEVICE); a cap the plan fits under gets to the device check."""
    xyz, tri = icosphere(2, 1.0)
    ctx = hps.hps_create(-1)
    try:
        hps.hps_set_mesh(ctx, xyz, tri)
        hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=300e6, leaf_max=16, device_mem_cap=1 << 20))
        with pytest.raises(hps.HpsError) as e:
            hps.hps_setup(ctx)
        assert e.value.status == -2 and "device_mem_cap" in str(e.value)
        hps.hps_build_hmatrix(ctx, hps.hps_params_default(freq_hz=300e6, leaf_max=16, device_mem_cap=1 << 40))
        with pytest.raises(hps.HpsError) as e:
            hps.hps_setup(ctx)
        assert e.value.status == -3
    finally:
        hps.hps_destroy(ctx)


def test_tuning_table_reader(tmp_path):
    """hps_set_tuning reads and checks the tile-shape table before it needs a
    device: a missing file is HPS_EIO, malformed JSON or bad entries
    HPS_EINVAL, a valid table reaches the device check (HPS_EDEVICE on a
    host-only context).  The committed table, if present, is valid."""
    ctx = hps.hps_create(-1)

    def status(text=None, path=None):
        if path is None:
            path = tmp_path / "t.json"
            path.write_text(text)
        try:
            hps.hps_set_tuning(ctx, str(path))
        except hps.HpsError as e:
            return e.status, str(e)
        return 0, ""

    try:
        assert status(path=tmp_path / "absent.json")[0] == -6
        for bad in ('{"entries": [', '[1, 2]', '{"entries": 3}', '{"entries": [{"class": "gemm", "shape": 0}]}',
                    '{"entries": [{"class": "sweep", "shape": 13}]}', '{"entries": [{"class": "sweep", "shape": 1.5}]}',
                    '{"entries": [{"class": "sweep", "shape": 0, "rhs_max": -1}]}', '{"entries": []} x',
                    '{"entries": [{"class": "sweep", "shape": 0, "precision": 3}]}',
                    '{"sweep_pull_kmax": -1, "entries": []}', '{"sweep_pull_kmax": 2.5, "entries": []}',
                    '{"sweep_pull_kmax": "all", "entries": []}'):
            st, msg = status(bad)
            assert st == -1, (bad, st, msg)
        ok = ('{"arch": "gfx950", "shapes": {"0": "32 x 32"}, "sweep_pull_kmax": 4096, "entries": ['
              '{"class": "sweep", "rhs_max": 64, "group_max": 48.5, "precision": 1, "shape": 3}, '
              '{"class": "schur", "rhs_max": null, "group_max": null, "shape": 2}], "measured": [1, true, null]}')
        st, msg = status(ok)
        assert st == -3 and "host-only" in msg, (st, msg)
        committed = os.path.join(ROOT, "paper_2109_04129_amd", "tuning", "gfx950.json")
        if os.path.exists(committed):
            assert status(path=committed)[0] == -3
    finally:
        hps.hps_destroy(ctx)
