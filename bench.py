"""Benchmark of the H-matrix power-series EFIE hot path on one MI355X.

A step is one pass of the whole hot path over the monostatic sweep of the
workload: hps_setup (symbolic phase, device LU/inverse of the scaled
diagonal blocks, right scaling coefficients, Schur updates with fill-in)
followed by hps_solve_planewaves (plane-wave RHS, forward sweep, D^-1, back
sweep, far field, second term, ratio, RCS).  The H-matrix (mesh, quadrature,
ACA) is built once before the timed region, as in the paper's tables, whose
"setup time" excludes the matrix fill.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

Prints one JSON line.  value = RHS solved per second over the timed steps
(setup included in every step); setup_s and solve-only RHS/s are reported
beside it.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "hbm": 8.0e12}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere_s5_790MHz")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rhs", type=int, default=8, help="RHS in the oracle's timed sample")
    return ap.parse_args()


def gpu_leg(args, w):
    import torch
    from paper_2109_04129_amd import hps

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    stream = torch.cuda.current_stream()
    ctx = hps.hps_create(0, stream.cuda_stream)
    hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
    p = hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"], aca_tol=w["aca_tol"], terms=2)
    t0 = time.perf_counter()
    hps.hps_build_hmatrix(ctx, p)
    build_s = time.perf_counter() - t0
    print("[bench] H-matrix built in %.1f s" % build_s, file=sys.stderr, flush=True)
    N = hps.hps_num_unknowns(ctx)
    khat, pol = w["khat"], w["pol"]
    R = len(khat)
    X = torch.zeros((R, N), dtype=torch.complex128, device="cuda")

    def step():
        ts = time.perf_counter()
        hps.hps_setup(ctx)
        tm = time.perf_counter()
        st, rcs, ratio = hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
        te = time.perf_counter()
        return tm - ts, te - tm, rcs, ratio

    for _ in range(args.warmup):
        step()
        print("[bench] warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    setup_t, solve_t = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a, b, rcs, ratio = step()
        setup_t.append(a)
        solve_t.append(b)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    stats = hps.hps_stats(ctx)
    hps.hps_destroy(ctx)
    return dict(N=N, R=R, total=total, setup=np.array(setup_t), solve=np.array(solve_t), rcs=rcs,
                ratio=ratio, stats=stats, build_s=build_s)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    from workloads import workload
    w = workload(args.workload)
    g = gpu_leg(args, w)
    R, K = g["R"], args.steps
    ms_per_step = 1e3 * g["total"] / K
    dev = g["stats"].get("device", {})
    out = {
        "metric": "RHS solved/sec + setup s at <=1e-3 rel err vs FP64; mixed/batched vs plain FP64",
        "value": R * K / g["total"],
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 (fp64)",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": g["N"], "rhs": R, "leaf_max": w["leaf_max"],
                   "aca_tol": w["aca_tol"], "freq_hz": w["freq_hz"], "form": "plain fp64", "terms": 2},
        "setup_s": float(np.median(g["setup"])),
        "solve_rhs_per_s": float(R / np.median(g["solve"])),
        "hmatrix_build_s": g["build_s"],
        "ratio_max": float(np.max(g["ratio"])),
        "device_stats": dev,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
