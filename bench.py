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
# dominant kernel: the grouped complex GEMM in subtract mode (Schur updates of
# the setup, forward and back sweeps of the solve), FP64 MFMA 16x16x4 (3M split)
DOMINANT = "gemm_sub"


def kernel_hash():
    """sha256 prefix of the grouped GEMM templates' source (k_gemm and the
    pipelined k_gemm_pipe, the functions themselves), to tie the counted
    traffic to them."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2109_04129_amd", "csrc", "device.hip")).read()
    h = hashlib.sha256()
    for name in ("void k_gemm(", "void k_gemm_pipe("):
        a = src.rindex("template <", 0, src.index(name))
        b = src.index("\n}\n", a) + 3
        h.update(src[a:b].encode())
    return h.hexdigest()[:16]


def counted_traffic(workload):
    """HBM bytes per k_gemm<1> launch from the committed rocprofv3 --pmc
    summary of this workload, or None if absent or taken on other code."""
    path = os.path.join(ROOT, "profiles", "k_gemm_%s.md" % workload)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_sha256_prefix"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    if vals.get("kernel_sha256_prefix") != kernel_hash():
        return None
    return float(vals["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in vals else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ellipsoid_4x2x1_300MHz")
    ap.add_argument("--leg-steps", type=int, default=1,
                    help="timed steps of each secondary leg (precision forms, CFIE, the second workload)")
    ap.add_argument("--second-workload", default="sphere_s5_790MHz",
                    help="secondary workload (plain, precision form and single-RHS legs); '' for none")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the precision-form legs")
    ap.add_argument("--no-cfie", action="store_true", help="skip the CFIE leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 32-ellipsoid batching leg")
    ap.add_argument("--cpu-sample-unknowns", type=int, default=16384,
                    help="largest cluster of the workload the oracle sample may take")
    ap.add_argument("--cpu-rhs", type=int, default=8, help="RHS in the oracle's timed sample")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 256 MiB device copy first (scale reference for HBM counters)")
    ap.add_argument("--only-headline", action="store_true",
                    help="headline leg only (for profiler runs): no secondary legs, no baseline")
    ap.add_argument("--batch-workload", default="ellipsoids32_600MHz")
    ap.add_argument("--only-single-rhs", action="store_true",
                    help="the single-RHS leg of --workload only (for profiler runs); prints its own JSON line")
    ap.add_argument("--tuning", default=None,
                    help="tile-shape table (JSON, as the autotuner writes) to use instead of the library's")
    ap.add_argument("--only-batch", action="store_true",
                    help="run only the batching leg (--batch-workload); prints its own JSON line")
    ap.add_argument("--leaf-study", action="store_true",
                    help="run only the leaf-size study (Sec. V.A): two-term and converged-series error against "
                         "the direct solution vs leaf size, EFIE and CFIE; prints its own JSON line")
    ap.add_argument("--scaling-study", action="store_true",
                    help="run only the scaling study (Sec. IV, Figs. 3 and 5): setup time, factor memory and "
                         "solve time vs unknowns on spheres of constant mesh density; prints its own JSON line")
    return ap.parse_args()


T_START = time.perf_counter()


def log(msg):
    print("[bench %7.1f s] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


def build_hmatrix(w, **extra):
    """The H-matrix of the workload, built once (near blocks and ACA sampling
    on the device, recompression on host threads; not timed as setup) and
    installed in every leg.  ``extra`` selects e.g. the CFIE formulation."""
    import torch
    from paper_2109_04129_amd import hps
    h = tuned(hps.hps_create(0, torch.cuda.current_stream().cuda_stream))
    try:
        set_mesh(hps, h, w)
        p = hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"], aca_tol=w["aca_tol"], verbose=1,
                                   **extra)
        t0 = time.perf_counter()
        hps.hps_build_hmatrix(h, p)
        build_s = time.perf_counter() - t0
        g = hps.hps_get_hmatrix(h)
        g["N"] = hps.hps_num_unknowns(h)
    finally:
        hps.hps_destroy(h)
    print("[bench] H-matrix built in %.1f s" % build_s, file=sys.stderr, flush=True)
    return g, build_s


def set_mesh(hps, ctx, w):
    (hps.hps_set_open_mesh if w.get("open") else hps.hps_set_mesh)(ctx, w["xyz"], w["tri"])


def install(hps, ctx, p, g):
    hps.hps_set_hmatrix(ctx, p, g["N"], g["perm"], g["group_ptr"], g["near_ts"], g["near_off"], g["near_vals"],
                        g["far_rng"], g["far_rank"], g["far_off"], g["far_uv"])


def copy_calib(args):
    """With --copy-calib: one 256 MiB device copy (a scale reference for the
    HBM byte counters of a profiler run)."""
    import torch
    if args.copy_calib:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)                   # 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        del src, dst


def gpu_leg(args, w, g, steps, warmup, precision=0, refine=0, reference_terms=None, extra=None,
            reference_tol=0.0, profile=True):
    """`steps` timed steps (hps_setup + the whole sweep's hps_solve_planewaves)
    after `warmup` untimed ones, unprofiled: solves are replayed from their
    captured graph, as in production.  Then, with `profile`, one more step
    with HIP events around every launch, for the per-kernel figures."""
    import torch
    from paper_2109_04129_amd import hps

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    copy_calib(args)
    stream = torch.cuda.current_stream()
    ctx = tuned(hps.hps_create(0, stream.cuda_stream))
    set_mesh(hps, ctx, w)
    kw = dict(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"], aca_tol=w["aca_tol"], terms=2, precision=precision,
              refine_passes=refine)
    kw.update(extra or {})
    p = hps.hps_params_default(**kw)
    install(hps, ctx, p, g)
    N = hps.hps_num_unknowns(ctx)
    khat, pol = w["khat"], w["pol"]
    R = len(khat)
    X = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
    status = []

    def step():
        ts = time.perf_counter()
        hps.hps_setup(ctx)
        tm = time.perf_counter()
        st, rcs, ratio = hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
        te = time.perf_counter()
        status.append(st)
        return tm - ts, te - tm, rcs, ratio

    for _ in range(warmup):
        step()
        log("warmup step done")
    torch.cuda.synchronize()
    setup_t, solve_t = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        a, b, rcs, ratio = step()
        setup_t.append(a)
        solve_t.append(b)
        log("step done")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    stats = hps.hps_stats(ctx)
    if profile:
        # one step with HIP events around every kernel launch (no graph
        # replay): per-kernel time, algorithmic flops and bytes, launch log
        hps.hps_profile(ctx, True)
        step()
        torch.cuda.synchronize()
        stats = hps.hps_stats(ctx)
        hps.hps_profile(ctx, False)
        log("profiled step done")
    hps.hps_destroy(ctx)
    err = None
    if reference_terms:
        # accuracy of this form against the plain FP64 path (parity-tested
        # against the oracle) on the same H-matrix, at the matching number of
        # series terms
        Xm = X.cpu().numpy()
        del X
        p.precision, p.refine_passes, p.terms, p.series_tol = 0, 0, reference_terms, reference_tol
        ref = tuned(hps.hps_create(0, stream.cuda_stream))
        set_mesh(hps, ref, w)
        install(hps, ref, p, g)
        hps.hps_setup(ref)
        Xr = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
        _, rcs_r, _ = hps.hps_solve_planewaves(ref, khat, pol, Xr.data_ptr())
        torch.cuda.synchronize()
        Xr = Xr.cpu().numpy()
        used = hps.hps_stats(ref).get("device", {}).get("terms_used")
        hps.hps_destroy(ref)
        log("reference solve done")
        err = {"terms_of_reference": reference_terms if reference_tol <= 0 else
               "adaptive to %g (%s terms)" % (reference_tol, used),
               "current_rel_err_max": float(np.max(np.linalg.norm(Xm - Xr, axis=1) / np.linalg.norm(Xr, axis=1))),
               "current_rel_err_median": float(np.median(np.linalg.norm(Xm - Xr, axis=1) /
                                                         np.linalg.norm(Xr, axis=1))),
               "rcs_db_err_max": float(np.max(np.abs(10 * np.log10(rcs / rcs_r))))}
    return dict(N=N, R=R, total=total, steps=steps, setup=np.array(setup_t), solve=np.array(solve_t), rcs=rcs,
                ratio=ratio, status=status[-1], stats=stats, err=err)


def single_rhs_leg(args, w, g, precision=0, reps=10):
    """One right-hand side (the sweep's first direction): the solve is a
    chain of matrix-vector products, bound by HBM bandwidth.  Device time of
    the solve (HIP events around its graph replay, median of `reps`), then
    one profiled solve for the per-kernel algorithmic bytes."""
    import torch
    from paper_2109_04129_amd import hps
    copy_calib(args)
    stream = torch.cuda.current_stream()
    ctx = tuned(hps.hps_create(0, stream.cuda_stream))
    try:
        set_mesh(hps, ctx, w)
        p = hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"], aca_tol=w["aca_tol"], terms=2,
                                   precision=precision, refine_passes=1 if precision else 0)
        install(hps, ctx, p, g)
        hps.hps_setup(ctx)
        N = hps.hps_num_unknowns(ctx)
        khat, pol = w["khat"][:1], w["pol"][:1]
        X = torch.zeros((1, N), dtype=torch.complex128, device="cuda")
        dev_ms, wall = [], []
        for i in range(reps + 2):          # direct launch, graph capture, then replays
            t0 = time.perf_counter()
            hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
            t1 = time.perf_counter()
            if i >= 2:
                dev_ms.append(hps.hps_stats(ctx)["device"]["times_ms"]["solve"])
                wall.append(t1 - t0)
        hps.hps_profile(ctx, True)
        hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
        torch.cuda.synchronize()
        st = hps.hps_stats(ctx)
        hps.hps_profile(ctx, False)
    finally:
        hps.hps_destroy(ctx)
    dev = st["device"]
    ks = dev.get("kernels", {})
    gemm_bytes = sum(ks.get(k, {}).get("bytes", 0.0) for k in ("gemm_store", "gemm_sub", "gemm_add"))
    gemm_ms = sum(ks.get(k, {}).get("ms", 0.0) for k in ("gemm_store", "gemm_sub", "gemm_add"))
    solve_ms = float(np.median(dev_ms))
    esz = 8 if precision else 16
    # SURVEY-style per-RHS count: every coefficient entry read in each of the
    # four sweeps, D^-1 twice, every stored far entry twice (one far product:
    # stage 1 and stage 2 each read every factor once)
    formula = esz * (4.0 * dev["n_U"] + 2.0 * dev["n_D"]) + (4 if precision else 16) * 2.0 * dev["far_elems"]
    k = ks.get("gemm_sub", {})
    sub = None
    if k.get("ms"):
        sub = {"kernel": "grouped GEMM, subtract mode (the sweeps; one column: k_gemv)", "bound": "hbm", "achieved": k["bytes"] / (k["ms"] * 1e-3) / 1e9,
               "peak": PEAK["hbm"] / 1e9, "unit": "GB/s",
               "frac": k["bytes"] / (k["ms"] * 1e-3) / PEAK["hbm"],
               "launches": k["launches"], "avg_launch_us": 1e3 * k["ms"] / k["launches"],
               "algorithmic_bytes_per_launch": k["bytes"] / k["launches"]}
    return {"workload": w["name"], "precision": precision, "N": N,
            "solve_ms_device": solve_ms, "solve_ms_wall": 1e3 * float(np.median(wall)),
            "rhs_per_s": 1e3 / solve_ms,
            "algorithmic_bytes": formula,
            "achieved_gb_s": formula / (solve_ms * 1e-3) / 1e9,
            "hbm_frac": formula / (solve_ms * 1e-3) / PEAK["hbm"],
            "gemm_launch_bytes": gemm_bytes, "gemm_launch_ms": gemm_ms,
            "gemm_achieved_gb_s": gemm_bytes / (gemm_ms * 1e-3) / 1e9 if gemm_ms else None,
            "dominant_kernel": sub}


def batch_leg(args):
    """Batching form: all problems in one context (every setup level and solve
    stage one launch for all of them) against the plain form, i.e. the same
    problems one context at a time, on the same H-matrices."""
    import torch
    from paper_2109_04129_amd import hps
    from workloads import batch_workload
    bw = batch_workload(args.batch_workload)
    P, R = len(bw["meshes"]), len(bw["khat"])
    khat, pol = bw["khat"], bw["pol"]
    stream = torch.cuda.current_stream().cuda_stream
    prm = hps.hps_params_default(freq_hz=bw["freq_hz"], leaf_max=bw["leaf_max"], aca_tol=bw["aca_tol"], terms=2)
    # H-matrices, one problem at a time (near blocks on the device, far blocks
    # on host threads; not timed as setup)
    parts, build_s = [], 0.0
    for p, (xyz, tri) in enumerate(bw["meshes"]):
        h = tuned(hps.hps_create(0, stream))
        hps.hps_set_mesh(h, xyz, tri)
        t0 = time.perf_counter()
        hps.hps_build_hmatrix(h, prm)
        build_s += time.perf_counter() - t0
        g = hps.hps_get_hmatrix(h)
        g["N"] = hps.hps_num_unknowns(h)
        parts.append(g)
        hps.hps_destroy(h)
        print("[bench] H-matrix %d/%d (%d unknowns) built" % (p + 1, P, g["N"]), file=sys.stderr, flush=True)
    Ns = [a["N"] for a in parts]
    NT = sum(Ns)

    def batch_ctx(precision, graphs=1):
        c = tuned(hps.hps_batch_create(P, 0, stream))
        for p, (xyz, tri) in enumerate(bw["meshes"]):
            hps.hps_batch_set_mesh(c, p, xyz, tri)
        prm.precision, prm.refine_passes, prm.graphs = precision, (1 if precision else 0), graphs
        for p, a in enumerate(parts):
            hps.hps_batch_set_hmatrix(c, p, prm, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"],
                                      a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        prm.precision, prm.refine_passes, prm.graphs = 0, 0, 1
        return c

    def timed(c, Xp, steps):
        su, so = [], []
        for _ in range(steps):
            ta = time.perf_counter()
            hps.hps_setup(c)
            tb = time.perf_counter()
            _, rcs, ratio = hps.hps_solve_planewaves(c, khat, pol, Xp.data_ptr())
            so.append(time.perf_counter() - tb)
            su.append(tb - ta)
        return np.array(su), np.array(so), rcs, ratio

    K = args.leg_steps

    def run_batch(c, precision, warm=1):
        Xb = torch.zeros(R * NT, dtype=torch.complex128, device="cuda")
        timed(c, Xb, warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        su, so, rcs, ratio = timed(c, Xb, K)
        torch.cuda.synchronize()
        return dict(total=time.perf_counter() - t0, setup=su, solve=so, rcs=rcs, ratio=ratio, X=Xb.cpu().numpy())

    ctx = batch_ctx(0)
    res = {0: run_batch(ctx, 0)}
    st = hps.hps_stats(ctx)
    hps.hps_destroy(ctx)
    print("[bench] batched FP64 done", file=sys.stderr, flush=True)
    # graphs = 2: the first setup runs eagerly and is recorded, the second
    # captures it; the timed setups replay that graph (every level recomputed
    # on the device from the installed values, no host scheduling)
    ctx = batch_ctx(0, graphs=2)
    res["g"] = run_batch(ctx, 0, warm=2)
    res["g"]["replays"] = hps.hps_stats(ctx)["device"].get("setup_replays")
    hps.hps_destroy(ctx)
    print("[bench] batched FP64 with setup graph done", file=sys.stderr, flush=True)
    ctx = batch_ctx(2)                       # precision form of the batch, same H-matrices
    res[2] = run_batch(ctx, 2)
    dev = dict(hps.hps_stats(ctx).get("device", {}))
    dev.pop("launch_log", None)
    hps.hps_destroy(ctx)
    print("[bench] batch legs done", file=sys.stderr, flush=True)
    # plain form: the same problems, one context after the other
    seq_total, seq_setup, seq_solve, worst, worst_db = 0.0, 0.0, 0.0, 0.0, 0.0
    off = 0
    for p, (xyz, tri) in enumerate(bw["meshes"]):
        c = tuned(hps.hps_create(0, stream))
        hps.hps_set_mesh(c, xyz, tri)
        a = parts[p]
        hps.hps_set_hmatrix(c, prm, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"], a["near_vals"],
                            a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        Xp = torch.zeros((R, Ns[p]), dtype=torch.complex128, device="cuda")
        timed(c, Xp, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        su, so, rcs_p, _ = timed(c, Xp, K)
        torch.cuda.synchronize()
        seq_total += time.perf_counter() - t0
        seq_setup += float(np.median(su))
        seq_solve += float(np.median(so))
        xp = Xp.cpu().numpy()
        xb = res[0]["X"][off * R:(off + Ns[p]) * R].reshape(R, Ns[p])
        worst = max(worst, float(np.max(np.linalg.norm(xb - xp, axis=1) / np.linalg.norm(xp, axis=1))))
        # the precision form (two-term series plus one residual pass) equals
        # the four-term series: its FP64 reference
        prm.terms = 4
        hps.hps_set_hmatrix(c, prm, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"], a["near_vals"],
                            a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        hps.hps_setup(c)
        _, rcs4, _ = hps.hps_solve_planewaves(c, khat, pol, Xp.data_ptr())
        torch.cuda.synchronize()
        prm.terms = 2
        x4 = Xp.cpu().numpy()
        xb = res[2]["X"][off * R:(off + Ns[p]) * R].reshape(R, Ns[p])
        e_p = float(np.max(np.linalg.norm(xb - x4, axis=1) / np.linalg.norm(x4, axis=1)))
        res[2]["err"] = max(res[2].get("err", 0.0), e_p)
        res[2].setdefault("per_problem", []).append(
            {"N": int(Ns[p]), "current_rel_err_vs_fp64_terms4": e_p,
             "ratio_max": float(np.max(res[0]["ratio"][p]))})
        worst_db = max(worst_db, float(np.max(np.abs(10 * np.log10(res[2]["rcs"][p] / rcs4)))))
        off += Ns[p]
        hps.hps_destroy(c)
        print("[bench] plain problem %d/%d done" % (p + 1, P), file=sys.stderr, flush=True)
    out = {"workload": bw["name"], "problems": P, "rhs_per_problem": R, "unknowns": NT,
           "unknowns_min_max": [min(Ns), max(Ns)], "hmatrix_build_s": build_s,
           "plain_sequential": {"rhs_per_s_step": P * R * K / seq_total, "setup_s": seq_setup,
                                "solve_rhs_per_s": P * R / seq_solve}}
    for form, name in ((0, "batched_fp64"), ("g", "batched_fp64_setup_graph"), (2, "batched_mixed_fp16_far")):
        r = res[form]
        out[name] = {"rhs_per_s_step": P * R * K / r["total"], "setup_s": float(np.median(r["setup"])),
                     "solve_rhs_per_s": P * R / float(np.median(r["solve"])),
                     "speedup_step_vs_plain": (P * R * K / r["total"]) / (P * R * K / seq_total)}
    out["batched_fp64"]["current_rel_err_vs_plain"] = worst
    g = out["batched_fp64_setup_graph"]
    g["setup"] = ("graphs = 2: the timed setups replay the first setup's launches from one captured HIP graph "
                  "(same structure; every level recomputed on the device)")
    g["setup_replays"] = res["g"]["replays"]
    g["currents_bitwise_equal_to_eager_batch"] = bool(np.array_equal(res["g"]["X"], res[0]["X"]))
    out["batched_mixed_fp16_far"]["current_rel_err_vs_fp64_terms4"] = res[2].get("err")
    out["batched_mixed_fp16_far"]["rcs_db_err_vs_fp64_terms4"] = worst_db
    out["batched_mixed_fp16_far"]["per_problem"] = res[2].get("per_problem")
    out["device_stats_fp16_form"] = {k: dev.get(k) for k in ("levels", "upper_blocks", "factor_bytes", "times_ms")}
    out["hmatrix"] = st.get("hmatrix")
    return out


def oracle_work(sizes, adj, order):
    """The oracle's own arithmetic, in complex multiply-adds, of its block
    elimination (eqs. 16-21, both triangles of every Schur update, as its
    schur_scaling does) in the given order, and of one right-hand side of its
    two-term solve without the far field: returns (setup MACs, 4 n_U + 2 n_D)."""
    nbr = {g: set(v) for g, v in adj.items()}
    done, setup, nU, nD = set(), 0.0, 0.0, 0.0
    for i in order:
        later = [j for j in nbr[i] if j not in done]
        ni = float(sizes[i])
        nF = float(sum(sizes[j] for j in later))
        setup += ni ** 3 + ni * ni * nF + ni * nF * nF
        nU += ni * nF
        nD += ni * ni
        for j in later:
            nbr[j].update(k for k in later if k != j)
        done.add(i)
    return setup, 4.0 * nU + 2.0 * nD


def cpu_leg(args, w):
    """The oracle, untuned, on the host cores, on a bounded sample of the
    same workload: the principal sub-H-matrix of one octree cluster (the
    largest with at most --cpu-sample-unknowns unknowns; its near and far
    blocks as the oracle builds them, untimed), its setup (timed) and the
    two-term solve of the first --cpu-rhs directions restricted to the
    cluster (timed).  Both times are scaled to the whole problem by the
    oracle's own operation counts (minimum-degree elimination of the full
    group graph vs the cluster's); far products by the summed far-block
    sizes.  The result is an extrapolation and is labelled so."""
    from threadpoolctl import threadpool_info
    from oracle.hmatrix import build_hmatrix_cluster
    from oracle.planewave import excitation
    from oracle.scaling import group_graph, min_degree_order, schur_scaling
    from oracle.series import PowerSeries
    workers = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    H, info = build_hmatrix_cluster(w["xyz"], w["tri"], w["freq_hz"], w["leaf_max"], w["aca_tol"],
                                    args.cpu_sample_unknowns, workers=workers)
    log("oracle cluster sample (%d of %d unknowns, %d groups) built in %.1f s"
        % (H.N, info["N"], H.M, time.perf_counter() - t0))
    t0 = time.perf_counter()
    order = min_degree_order(group_graph(H))
    S = schur_scaling(H, order)
    setup_s = time.perf_counter() - t0
    log("oracle sample setup %.1f s" % setup_s)
    R = args.cpu_rhs
    b = excitation(info["rwg"], w["freq_hz"], w["khat"][:R], w["pol"][:R])[H.rwg_index]
    t0 = time.perf_counter()
    PowerSeries(H, S).solve(b, 2)
    solve_s = time.perf_counter() - t0
    log("oracle sample solve %.2f s" % solve_s)
    # operation counts of the sample and of the whole problem, oracle's order
    gs = [int(hi - lo) for lo, hi in H.groups]
    su_s, near_s = oracle_work(gs, group_graph(H), order)
    adj = {g: set() for g in range(len(info["leaf_sizes"]))}
    for t, u in info["near_pairs"]:
        if t != u:
            adj[t].add(u)
            adj[u].add(t)
    su_f, near_f = oracle_work(info["leaf_sizes"], adj, min_degree_order(adj))
    far_s = float(sum(2 * U.shape[1] * (U.shape[0] + V.shape[0]) for *_, U, V in H.far))
    msum_s = float(sum((thi - tlo) + (shi - slo) for tlo, thi, slo, shi, _, _ in H.far))
    msum_f = float(sum(m + n for m, n in info["far_sizes"]))
    far_f = far_s * msum_f / max(msum_s, 1.0)
    setup_full = setup_s * su_f / su_s
    per_rhs_full = solve_s / R * (near_f + far_f) / (near_s + far_s)
    RT = len(w["khat"])
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": RT / (setup_full + RT * per_rhs_full), "unit": "RHS/s", "cores": threads, "kind": "oracle",
            "sample": ("extrapolation: the oracle (untuned) on the principal sub-H-matrix of one octree cluster "
                       "of the same workload (%d of %d unknowns, %d of %d groups), setup timed %.1f s and the "
                       "two-term solve of the first %d of its %d directions timed %.2f s, scaled by the oracle's "
                       "own operation counts (minimum-degree block elimination of the full group graph: setup "
                       "x%.1f, near solve per RHS x%.1f; far products by summed far-block sizes); value = "
                       "whole-sweep RHS / (extrapolated setup + %d x extrapolated per-RHS solve)"
                       % (H.N, info["N"], H.M, len(info["leaf_sizes"]), setup_s, R, RT, solve_s, su_f / su_s,
                          near_f / near_s, RT)),
            "extrapolated_setup_s": setup_full, "extrapolated_solve_rhs_per_s": 1.0 / per_rhs_full,
            "sample_setup_s": setup_s, "sample_solve_s": solve_s, "sample_unknowns": H.N,
            "host_cpus": os.cpu_count()}


def roofline_from(stats, steps=1):
    """Roofline object of the dominant kernel (k_gemm<1>: Schur updates and
    sweeps, complex FP64 on MFMA) from one profiled step.  Setup Schur
    updates and multi-RHS sweeps are dense contractions: bound = FP64 MFMA;
    the per-launch algorithmic bytes are reported beside it."""
    dev = dict(stats.get("device", {}))
    log_ = dev.pop("launch_log", None) or []
    k = dev.get("kernels", {}).get(DOMINANT, {})
    if not (k.get("ms") and k.get("bytes")):
        return None, dev
    classes = []
    sub = [x for x in log_ if x[0] == 1 and len(x) >= 5]
    for lo, hi in ((0, 1e7), (1e7, 1e8), (1e8, 1e9), (1e9, float("inf"))):
        sel = [x for x in sub if lo <= x[3] < hi]
        if sel:
            b, f, t = sum(x[3] for x in sel), sum(x[2] for x in sel), sum(x[4] for x in sel) * 1e-3
            classes.append({"bytes_per_launch": [lo, hi if hi != float("inf") else None],
                            "launches_per_step": len(sel) / steps, "ms_per_step": 1e3 * t / steps,
                            "achieved_gb_s": b / t / 1e9, "hbm_frac": b / t / PEAK["hbm"],
                            "achieved_tflops": f / t / 1e12, "intensity_flop_per_byte": f / b})
    sec = k["ms"] * 1e-3
    flop_rate, byte_rate = k["flops"] / sec, k["bytes"] / sec
    return {"kernel": "grouped complex GEMM on FP64 MFMA, subtract mode (k_gemm / k_gemm_pipe by tile shape)",
            "bound": "mfma",
            "achieved": flop_rate / 1e12, "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s",
            "frac": flop_rate / PEAK["fp64"],
            "flops_per_launch": k["flops"] / k["launches"],
            "algorithmic_bytes_per_launch": k["bytes"] / k["launches"],
            "achieved_gb_s_algorithmic": byte_rate / 1e9, "hbm_frac_algorithmic": byte_rate / PEAK["hbm"],
            "intensity_flop_per_byte": k["flops"] / k["bytes"], "ridge_flop_per_byte": PEAK["fp64"] / PEAK["hbm"],
            "launches_per_step": k["launches"] / steps, "avg_launch_us": 1e3 * k["ms"] / k["launches"],
            "by_launch_size": classes}, dev


def form_summary(gm, base):
    """Figures of one leg, with its speed against the plain FP64 leg."""
    rate = gm["R"] * gm["steps"] / gm["total"]
    return {"rhs_per_s_step": rate, "ms_per_step": 1e3 * gm["total"] / gm["steps"], "steps": gm["steps"],
            "setup_s": float(np.median(gm["setup"])),
            "solve_rhs_per_s": float(gm["R"] / np.median(gm["solve"])),
            "speedup_step_vs_plain_fp64": rate / (base["R"] * base["steps"] / base["total"]),
            "speedup_solve_vs_plain_fp64": float(np.median(base["solve"]) / np.median(gm["solve"])),
            "ratio_max": float(np.max(gm["ratio"])), "status": gm["status"],
            "accuracy_vs_fp64": gm["err"]}


def precision_legs(args, w, hm, base, variants=((1, "bf16_far"), (2, "fp16_far"))):
    """The precision form (FP32 solve operands on MFMA, 16-bit far factors
    with per-block FP32 scale, FP64 setup) with one FP32 residual pass, i.e.
    the four-term series: BF16 far factors (the configured form) and FP16;
    accuracy against the FP64 four-term series on the same H-matrix."""
    forms = {}
    for prec, name in variants:
        gm = gpu_leg(args, w, hm, args.leg_steps, 1, precision=prec, refine=1, reference_terms=4, profile=False)
        forms[name] = dict(form_summary(gm, base), residual_passes=1)
        log("precision form %s done" % name)
    return {"form": "FP32 near operands on MFMA, 16-bit far factors with per-block FP32 scale, FP64 setup, "
                    "one FP32 residual pass (= four-term series), against the FP64 four-term series",
            "variants": forms}


def cfie_leg(args, w):
    """CFIE of eq. (8), alpha = 0.5, on the same mesh: its own H-matrix
    (both orders of every block), left and right coefficients; accuracy of
    the two-term series against the converged series."""
    extra = {"formulation": 1, "cfie_alpha": 0.5}
    hc, bc = build_hmatrix(w, **extra)
    gc = gpu_leg(args, w, hc, args.leg_steps, 1, extra=extra, reference_terms=60, reference_tol=1e-10, profile=False)
    dc = gc["stats"].get("device", {})
    out = {"form": "CFIE alpha 0.5, plain fp64, two terms", "workload": w["name"],
           "rhs_per_s_step": gc["R"] * gc["steps"] / gc["total"],
           "ms_per_step": 1e3 * gc["total"] / gc["steps"],
           "setup_s": float(np.median(gc["setup"])),
           "solve_rhs_per_s": float(gc["R"] / np.median(gc["solve"])),
           "hmatrix_build_s": bc, "ratio_max": float(np.max(gc["ratio"])),
           "ratio_median": float(np.median(gc["ratio"])),
           "two_terms_vs_converged_series": gc["err"],
           "factor_bytes": dc.get("factor_bytes"), "upper_blocks": dc.get("upper_blocks")}
    ea = dict(extra, terms=40, series_tol=1e-4)
    ga = gpu_leg(args, w, hc, args.leg_steps, 1, extra=ea, reference_terms=60, reference_tol=1e-10, profile=False)
    out["adaptive_series_1e-4"] = {
        "rhs_per_s_step": ga["R"] * ga["steps"] / ga["total"],
        "solve_rhs_per_s": float(ga["R"] / np.median(ga["solve"])),
        "terms_used": ga["stats"].get("device", {}).get("terms_used"),
        "vs_converged_series": ga["err"]}
    return out


def secondary_leg(args, name):
    """The 30,720-unknown sphere: plain FP64 step, precision forms, R = 1."""
    from workloads import workload
    w = workload(name)
    w["name"] = name
    hm, build_s = build_hmatrix(w)
    g = gpu_leg(args, w, hm, max(args.leg_steps, 3), 1)
    roof, dev = roofline_from(g["stats"])
    out = {"workload": name, "N": g["N"], "rhs": g["R"], "hmatrix_build_s": build_s,
           "rhs_per_s_step": g["R"] * g["steps"] / g["total"], "ms_per_step": 1e3 * g["total"] / g["steps"],
           "setup_s": float(np.median(g["setup"])), "solve_rhs_per_s": float(g["R"] / np.median(g["solve"])),
           "ratio_max": float(np.max(g["ratio"])), "roofline": roof,
           "device_stats": {k: dev.get(k) for k in ("levels", "upper_blocks", "n_U", "n_D", "setup_flops",
                                                     "factor_bytes", "far_elems")}}
    if not args.no_mixed:
        out["precision_form"] = precision_legs(args, w, hm, g)
    out["single_rhs"] = single_rhs_leg(args, w, hm)
    log("secondary workload done")
    if not args.no_cfie:
        out["cfie_form"] = cfie_leg(args, w)
        log("CFIE leg done")
    return out


def leaf_study(args):
    """Sec. V.A (Fig. 4): accuracy of the two-term series against the direct
    solution of the same discretisation as the leaves grow, with the eq. (45)
    ratio.  Sphere r = 1 m, icosphere subdivision 5 (30,720 unknowns) at
    800 MHz (edges about lambda/10, the sphere 5.3 wavelengths across).  The
    direct solution is the library's own with eta = 0 (nothing admissible:
    Z_F = 0, every leaf pair a near block, so the setup is a block LDL^T of
    the full MoM matrix and one series term solves exactly), on cells of at
    least 0.5 m cut into pivots of at most 128 unknowns.  Leaves by unknown
    count (octree split while a cell has more than leaf_max) and by
    electrical size (leaf_max 16, cells never narrower than leaf_box_min).
    Error = max over RHS of ||x - x_dir|| / ||x_dir||, for two terms and for
    the series run until ||it_t|| / ||it_0|| < 1e-8 (at most 60 terms; it
    only converges where the ratio is below one)."""
    import torch
    from paper_2109_04129_amd import hps
    from workloads import icosphere, monostatic_angles
    freq = 800e6
    lam = 299792458.0 / freq
    xyz, tri = icosphere(5, 1.0)
    khat, pol = monostatic_angles([0.0, 45.0, 90.0, 135.0, 180.0], [0.0, 0.0, 0.0, 0.0, 0.0])
    R = len(khat)
    stream = torch.cuda.current_stream().cuda_stream

    def solve(form, leaf, box, eta, terms, tol=0.0):
        ctx = tuned(hps.hps_create(0, stream))
        try:
            hps.hps_set_mesh(ctx, xyz, tri)
            p = hps.hps_params_default(freq_hz=freq, leaf_max=leaf, aca_tol=1e-3, terms=terms, series_tol=tol,
                                       leaf_box_min=box, eta=eta, formulation=form, cfie_alpha=0.5)
            hps.hps_build_hmatrix(ctx, p)
            hps.hps_setup(ctx)
            N = hps.hps_num_unknowns(ctx)
            X = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
            st, rcs, ratio = hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
            torch.cuda.synchronize()
            d = hps.hps_stats(ctx)
            dev = d.get("device", {})
            return X.cpu().numpy(), ratio, rcs, dict(groups=(d.get("hmatrix") or {}).get("groups"), terms_used=dev.get("terms_used"),
                                                     far_blocks=(d.get("hmatrix") or {}).get("far_blocks"))
        finally:
            hps.hps_destroy(ctx)

    def err(x, ref):
        return float(np.max(np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)))

    rows = []
    cases = [("count", lf, 0.0) for lf in (16, 32, 64, 128)] + \
            [("box", 16, f * lam) for f in (0.15, 0.3, 0.6, 1.2)]
    for form, fname in ((0, "EFIE"), (1, "CFIE alpha 0.5")):
        xd, _, rcs_d, _ = solve(form, 128, 0.5, 0.0, 1)
        log("leaf study %s: direct solution done" % fname)
        for kind, leaf, box in cases:
            x2, ratio, rcs2, info = solve(form, leaf, box, 2.0, 2)
            xc, _, _, infoc = solve(form, leaf, box, 2.0, 60, 1e-8)
            rows.append({"formulation": fname, "leaves": kind, "leaf_max": leaf, "leaf_box_min_lambda": box / lam,
                         "groups": info["groups"], "far_blocks": info["far_blocks"],
                         "mean_unknowns_per_group": float(xd.shape[1]) / max(info["groups"] or 1, 1),
                         "ratio_eq45_max": float(np.max(ratio)), "ratio_eq45_median": float(np.median(ratio)),
                         "two_term_err_vs_direct": err(x2, xd),
                         "two_term_rcs_db_err_max": float(np.max(np.abs(10 * np.log10(rcs2 / rcs_d)))),
                         "series_1e-8_err_vs_direct": err(xc, xd), "series_terms_used": infoc["terms_used"]})
            log("leaf study %s %s %s done" % (fname, kind, leaf if kind == "count" else box / lam))
    return {"study": "leaf size (Sec. V.A, Fig. 4 metric)", "workload": "sphere r=1 m, icosphere subdiv 5, "
            "30,720 unknowns, 800 MHz (lambda %.4f m), ACA 1e-3, 5 monostatic RHS theta = 0..180 step 45" % lam,
            "direct": "library, eta = 0 on cells of at least 0.5 m cut into pivots of at most 128 unknowns "
                      "(no far blocks: block LDL^T of the full MoM matrix, one term)",
            "rows": rows}


def scaling_study(args):
    """Sec. IV (eqs. 46-56) and Figs. 3 and 5: setup time and the memory of the
    scaling coefficients and scaled near-field blocks grow as O(N), the
    solution as O(N log N).  Spheres of constant mesh density (icosphere
    subdivision s, radius 2^(s-5) m, 790 MHz: the 30,720-unknown sphere's
    edge length at every size), leaf <= 128, ACA 1e-3, plain FP64, two terms.
    Per size: the setup (mean of two after a warm-up), the factor panels'
    bytes, a 32-RHS solve per RHS and a one-RHS solve (means of two after a
    warm-up, device work synchronised); the log-log slopes over the sizes."""
    import torch
    from paper_2109_04129_amd import hps
    from workloads import icosphere, monostatic_angles
    freq = 790e6
    stream = torch.cuda.current_stream().cuda_stream
    rows = []
    for sub in (3, 4, 5, 6):
        xyz, tri = icosphere(sub, 2.0 ** (sub - 5))
        ctx = tuned(hps.hps_create(0, stream))
        try:
            hps.hps_set_mesh(ctx, xyz, tri)
            p = hps.hps_params_default(freq_hz=freq, leaf_max=128, aca_tol=1e-3, terms=2)
            t0 = time.perf_counter()
            hps.hps_build_hmatrix(ctx, p)
            t_build = time.perf_counter() - t0
            N = hps.hps_num_unknowns(ctx)

            def timed(fn, reps=2):
                fn()
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(reps):
                    fn()
                torch.cuda.synchronize()
                return (time.perf_counter() - t) / reps

            t_setup = timed(lambda: hps.hps_setup(ctx))
            res = {}
            for R in (32, 1):
                th = np.linspace(0.0, 180.0, R) if R > 1 else np.array([90.0])
                khat, pol = monostatic_angles(th, np.zeros_like(th))
                X = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
                res[R] = timed(lambda: hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr()))
            d = hps.hps_stats(ctx)
            dev = d.get("device", {})
            rows.append({"subdivision": sub, "radius_m": 2.0 ** (sub - 5), "N": int(N),
                         "groups": (d.get("hmatrix") or {}).get("groups"),
                         "hmatrix_build_s": t_build, "setup_s": t_setup,
                         "factor_gb": dev.get("factor_bytes", 0) / 1e9,
                         "solve_ms_per_rhs_32": 1e3 * res[32] / 32, "solve_ms_1rhs": 1e3 * res[1]})
            log("scaling study: N = %d done (setup %.3f s)" % (N, t_setup))
        finally:
            hps.hps_destroy(ctx)
    lg = np.log([r["N"] for r in rows])

    def slope(key):
        return float(np.polyfit(lg, np.log([r[key] for r in rows]), 1)[0])

    return {"study": "scaling (Sec. IV, Figs. 3 and 5)",
            "workload": "spheres of constant mesh density: icosphere subdivision 3-6, radius 2^(s-5) m, 790 MHz, "
                        "leaf <= 128, ACA 1e-3, plain FP64, two terms",
            "rows": rows,
            "loglog_slope_vs_N": {k: slope(k) for k in ("setup_s", "factor_gb", "solve_ms_per_rhs_32",
                                                       "solve_ms_1rhs")}}


TUNING_PATH = None


def tuned(ctx):
    """A new context with the --tuning table in place of the library's own."""
    if TUNING_PATH:
        from paper_2109_04129_amd import hps
        hps.hps_set_tuning(ctx, TUNING_PATH)
    return ctx


def main():
    global TUNING_PATH
    args = parse()
    TUNING_PATH = args.tuning
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.leaf_study:
        print(json.dumps(leaf_study(args)), flush=True)
        return
    if args.scaling_study:
        print(json.dumps(scaling_study(args)), flush=True)
        return
    if args.only_batch:
        print(json.dumps(batch_leg(args)), flush=True)
        return
    if args.only_single_rhs:
        from workloads import workload
        w = workload(args.workload)
        w["name"] = args.workload
        hm, _ = build_hmatrix(w)
        print(json.dumps(single_rhs_leg(args, w, hm)), flush=True)
        return
    from workloads import workload
    w = workload(args.workload)
    w["name"] = args.workload
    hm, build_s = build_hmatrix(w)
    log("workload %s: %d unknowns, %d RHS" % (args.workload, hm["N"], len(w["khat"])))
    g = gpu_leg(args, w, hm, args.steps, args.warmup)
    log("headline leg done")
    R, K = g["R"], args.steps
    roofline, dev = roofline_from(g["stats"])
    if roofline is not None:
        roofline["traffic"] = counted_traffic(args.workload)
    single = mixed = second = batch = cpu = None
    if not args.only_headline:
        single = single_rhs_leg(args, w, hm)
        log("single-RHS leg done")
        if not args.no_mixed:
            mixed = precision_legs(args, w, hm, g, variants=((1, "bf16_far"),))
        del hm
        if args.second_workload:
            second = secondary_leg(args, args.second_workload)
        if not args.no_batch:
            batch = batch_leg(args)
            log("batching leg done")
        if not args.no_cpu_baseline:
            cpu = cpu_leg(args, w)
    out = {
        "metric": "RHS solved/sec + setup s at <=1e-3 rel err vs FP64; mixed/batched vs plain FP64",
        "value": R * K / g["total"],
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * g["total"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": g["N"], "rhs": R, "leaf_max": w["leaf_max"],
                   "aca_tol": w["aca_tol"], "freq_hz": w["freq_hz"], "form": "plain fp64", "terms": 2},
        "setup_s": float(np.median(g["setup"])),
        "solve_rhs_per_s": float(R / np.median(g["solve"])),
        "timing": "value and ms_per_step: the K timed steps without per-launch events (solves replayed "
                  "from their captured HIP graph); roofline: one further step with HIP events around "
                  "every launch",
        "hmatrix_build_s": build_s,
        "status": g["status"],
        "ratio_max": float(np.max(g["ratio"])),
        "ratio_ge_warn_fraction": float(np.mean(np.asarray(g["ratio"]) >= 0.1)),
        "roofline": roofline,
        "single_rhs": single,
        "precision_form": mixed,
        "batching_form": batch,
        "second_workload": second,
        "cpu_baseline": cpu,
        "device_stats": dev,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
