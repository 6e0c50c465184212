"""Autotuner of the grouped complex GEMM's tile shapes (the batching form's
"tile shapes chosen by an autotuner").

    python -m paper_2109_04129_amd.autotune [--workloads A B ...] [--rhs 1 32 0] [--out PATH]

For each workload the library builds the H-matrix once on the device; then

* setup: hps_setup is timed (wall clock, median of --reps, no per-launch
  events) with the Schur-update class forced to each tile shape in turn;
* solve: for each solve form (FP64; the FP32 form with BF16 far factors and
  its residual pass, whose kernels the FP16 form shares), each RHS count
  (0 = the workload's whole sweep) and each shape, one solve with every
  solve class forced to that shape runs with per-launch HIP events; the
  launch log's tuning class then gives each class's summed kernel time
  under each shape.

Each class takes its fastest shape.  The table (JSON, read by hps_set_tuning
and loaded by hps_create from tuning/gfx950.json next to libhps.so) holds one
entry per class, RHS bucket and mean-pivot-size bucket: buckets meet at the
geometric mean of neighbouring tuned RHS counts and at the arithmetic mean
of neighbouring workloads' mean pivot sizes; the last bucket is open.  The
measurements are kept in the file beside the entries.  All shapes give
bitwise the same results, so the table changes speed only.
"""

import argparse
import json
import math
import os
import sys
import tempfile
import time

CLASSES = ["sweep", "dinv", "far1", "far2", "near", "schur"]
SOLVE_CLASSES = CLASSES[:5]
SHAPES = 13
SHAPE_DOC = {0: "32 x 32 tile, waves 2 x 2 of 16 x 16 (FP64 built for 4 waves per SIMD)", 1: "32 x 64 tile, waves 2 x 2 of 16 x 32",
             2: "32 x 64 tile, waves 1 x 4 of 32 x 16", 3: "32 x 128 tile, waves 1 x 4 of 32 x 32",
             4: "32 x 128 tile, waves 2 x 2 of 16 x 64",
             5: "32 x 64 tile, waves 1 x 4 of 32 x 16, operands staged in LDS (FP64; FP32 takes shape 2)",
             6: "one-column FP64 solves: vector-ALU matrix-vector kernel (else shape 0)",
             7: "as 2, built for 3 waves per SIMD (FP64; FP32 takes 2)",
             8: "as 1, built for 3 waves per SIMD (FP64; FP32 takes 1)",
             9: "as 0, built for 5 waves per SIMD (FP64; FP32 takes 0)",
             10: "as 3, built for 4 waves per SIMD (FP32; FP64 takes 3)",
             11: "as 2, full 16-k chunks staged in LDS one chunk ahead by direct-to-LDS loads, target tile in LDS "
                 "(FP64; FP32 with FP32 factors: the pipelined FP32 kernel; 16-bit factors: 2)",
             12: "as 11, target tile fetched after the products (FP32 as for 11)"}
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning", "gfx950.json")


def _log(msg):
    print("[autotune] " + msg, file=sys.stderr, flush=True)


def _table(entries):
    fd, path = tempfile.mkstemp(suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump({"entries": entries}, f)
    return path


def _context(hps, torch, w, hm=None, precision=0):
    """A device context on the workload's mesh with its H-matrix: built on
    the device when hm is None, else installed from hm."""
    ctx = hps.hps_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        (hps.hps_set_open_mesh if w.get("open") else hps.hps_set_mesh)(ctx, w["xyz"], w["tri"])
        p = hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"], aca_tol=w["aca_tol"], terms=2,
                                   precision=precision, refine_passes=1 if precision else 0)
        if hm is None:
            hps.hps_build_hmatrix(ctx, p)
        else:
            hps.hps_set_hmatrix(ctx, p, hm["N"], hm["perm"], hm["group_ptr"], hm["near_ts"], hm["near_off"],
                                hm["near_vals"], hm["far_rng"], hm["far_rank"], hm["far_off"], hm["far_uv"])
        return ctx
    except BaseException:
        hps.hps_destroy(ctx)
        raise


def tune_workload(name, rhs_list, reps, precisions=(0, 1)):
    import numpy as np
    import torch
    from paper_2109_04129_amd import hps
    from workloads import workload
    w = workload(name)
    tmp = []

    def table(entries):
        path = _table(entries)
        tmp.append(path)
        return path

    try:
        # setup (FP64 in every form): the Schur class, by setup wall time
        ctx = _context(hps, torch, w)
        try:
            N = hps.hps_num_unknowns(ctx)
            hm = hps.hps_get_hmatrix(ctx)
            hm["N"] = N
            hps.hps_set_tuning(ctx, None)
            hps.hps_setup(ctx)
            groups = hps.hps_stats(ctx)["device"]["groups"]
            g = N / groups
            _log("%s: %d unknowns, %d pivot groups (mean %.1f)" % (name, N, groups, g))
            res = {"workload": name, "N": N, "pivot_groups": groups, "mean_pivot": g, "setup_ms": {},
                   "solve_ms": {}}
            for sh in range(SHAPES):
                hps.hps_set_tuning(ctx, table([{"class": "schur", "shape": sh}]))
                hps.hps_setup(ctx)
                ts = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    hps.hps_setup(ctx)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                res["setup_ms"][sh] = 1e3 * float(np.median(ts))
                _log("%s setup, Schur shape %d: %.2f ms" % (name, sh, res["setup_ms"][sh]))
        finally:
            hps.hps_destroy(ctx)
        res["best"] = {"schur": min(res["setup_ms"], key=res["setup_ms"].get), "solve": {}}
        # solve classes, per solve precision (0: FP64; 1: the FP32 form with
        # BF16 far factors and its residual pass) and RHS count, by summed
        # per-class launch time (HIP events)
        Rs = sorted(set(len(w["khat"]) if r == 0 else r for r in rhs_list))
        for prec in precisions:
            ctx = _context(hps, torch, w, hm, prec)
            try:
                hps.hps_setup(ctx)
                for R in Rs:
                    idx = np.arange(R) % len(w["khat"])
                    khat, pol = w["khat"][idx], w["pol"][idx]
                    X = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
                    per = {c: {} for c in SOLVE_CLASSES}
                    for sh in range(SHAPES):
                        hps.hps_set_tuning(ctx, table([{"class": c, "shape": sh} for c in SOLVE_CLASSES]))
                        hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())     # warm
                        hps.hps_profile(ctx, True)
                        hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
                        torch.cuda.synchronize()
                        log = hps.hps_stats(ctx)["device"].get("launch_log", [])
                        hps.hps_profile(ctx, False)
                        for c, cname in enumerate(SOLVE_CLASSES):
                            per[cname][sh] = sum(x[4] for x in log if len(x) >= 6 and x[5] == c)
                        _log("%s precision %d R=%d shape %d: %s" % (
                            name, prec, R, sh, ", ".join("%s %.2f ms" % (c, per[c][sh]) for c in SOLVE_CLASSES)))
                    res["solve_ms"]["%d/%d" % (prec, R)] = per
                    # a class with no launches in this form keeps shape 0
                    res["best"]["solve"].setdefault(prec, {})[R] = {
                        c: (min(per[c], key=per[c].get) if any(per[c].values()) else 0) for c in SOLVE_CLASSES}
                    del X
            finally:
                hps.hps_destroy(ctx)
        return res
    finally:
        for path in tmp:
            try:
                os.remove(path)
            except OSError:
                pass


def make_table(results):
    """Entries in match order: workloads by mean pivot size, then solve
    precision, then RHS buckets; the FP32 tuning (BF16 far factors) also
    serves the FP16 form, which runs the same kernels."""
    results = sorted(results, key=lambda r: r["mean_pivot"])
    entries = []
    for i, r in enumerate(results):
        gmax = None if i + 1 == len(results) else 0.5 * (r["mean_pivot"] + results[i + 1]["mean_pivot"])
        for prec, best in sorted(r["best"]["solve"].items()):
            Rs = sorted(best)
            for pr in ((0,) if prec == 0 else (1, 2)):
                for j, R in enumerate(Rs):
                    rmax = None if j + 1 == len(Rs) else int(math.floor(math.sqrt(R * Rs[j + 1])))
                    for c in SOLVE_CLASSES:
                        entries.append({"class": c, "rhs_max": rmax, "group_max": gmax, "precision": pr,
                                        "shape": int(best[R][c])})
        entries.append({"class": "schur", "rhs_max": None, "group_max": gmax, "shape": int(r["best"]["schur"])})
    return entries


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", nargs="+", default=["sphere_s5_790MHz", "ellipsoid_4x2x1_300MHz"])
    ap.add_argument("--rhs", nargs="+", type=int, default=[1, 32, 0],
                    help="RHS counts to tune the solve at (0 = the workload's whole sweep)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--precisions", nargs="+", type=int, default=[0, 1],
                    help="solve forms to tune (0 FP64, 1 FP32 with BF16 far factors; 1 also serves 2)")
    ap.add_argument("--out", default=DEFAULT_OUT)
    a = ap.parse_args()
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    results = [tune_workload(n, a.rhs, a.reps, tuple(a.precisions)) for n in a.workloads]
    table = {"arch": "gfx950", "shapes": SHAPE_DOC,
             "note": "written by paper_2109_04129_amd/autotune.py; entries match in order (first match wins)",
             "entries": make_table(results), "measured": results}
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    tmp = a.out + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1)
    os.replace(tmp, a.out)
    _log("wrote %s (%d entries)" % (a.out, len(table["entries"])))
    print(json.dumps({"out": a.out, "entries": table["entries"]}))


if __name__ == "__main__":
    main()
