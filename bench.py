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
    """sha256 prefix of the k_gemm source, to tie the counted traffic to it."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2109_04129_amd", "csrc", "device.hip")).read()
    a = src.rindex("template <", 0, src.index("void k_gemm("))
    b = src.index("// ------------------------------------------------------------------", a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


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
    ap.add_argument("--workload", default="sphere_s5_790MHz")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the precision-form leg")
    ap.add_argument("--no-cfie", action="store_true", help="skip the CFIE leg")
    ap.add_argument("--cpu-rhs", type=int, default=8, help="RHS in the oracle's timed sample")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 256 MiB device copy first (scale reference for HBM counters)")
    ap.add_argument("--batch", action="store_true",
                    help="also run the batching form on the 32-ellipsoid workload (host H-matrix build "
                         "of 735k unknowns takes a few minutes)")
    ap.add_argument("--batch-workload", default="ellipsoids32_600MHz")
    return ap.parse_args()


def build_hmatrix(w, **extra):
    """The H-matrix of the workload, built once (near blocks and ACA sampling
    on the device, recompression on host threads; not timed as setup) and
    installed in every leg.  ``extra`` selects e.g. the CFIE formulation."""
    import torch
    from paper_2109_04129_amd import hps
    h = hps.hps_create(0, torch.cuda.current_stream().cuda_stream)
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


def gpu_leg(args, w, g, precision=0, refine=0, reference_terms=None, extra=None, reference_tol=0.0):
    import torch
    from paper_2109_04129_amd import hps

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.copy_calib:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)                   # 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.current_stream()
    ctx = hps.hps_create(0, stream.cuda_stream)
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
    hps.hps_profile(ctx, True)          # HIP events around every kernel launch of the timed steps
    setup_t, solve_t = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a, b, rcs, ratio = step()
        setup_t.append(a)
        solve_t.append(b)
        print("[bench] step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    stats = hps.hps_stats(ctx)
    # the same steps without per-launch events (solves replayed from their
    # captured graph, the production mode); reported beside the timed value
    hps.hps_profile(ctx, False)
    step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    total_unprofiled = time.perf_counter() - t1
    hps.hps_destroy(ctx)
    err = None
    if reference_terms:
        # accuracy of this form against the plain FP64 path (parity-tested
        # against the oracle) on the same H-matrix, at the matching number of
        # series terms
        Xm = X.cpu().numpy()
        del X
        p.precision, p.refine_passes, p.terms, p.series_tol = 0, 0, reference_terms, reference_tol
        ref = hps.hps_create(0, stream.cuda_stream)
        set_mesh(hps, ref, w)
        install(hps, ref, p, g)
        hps.hps_setup(ref)
        Xr = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
        _, rcs_r, _ = hps.hps_solve_planewaves(ref, khat, pol, Xr.data_ptr())
        torch.cuda.synchronize()
        Xr = Xr.cpu().numpy()
        used = hps.hps_stats(ref).get("device", {}).get("terms_used")
        hps.hps_destroy(ref)
        err = {"terms_of_reference": reference_terms if reference_tol <= 0 else
               "adaptive to %g (%s terms)" % (reference_tol, used),
               "current_rel_err_max": float(np.max(np.linalg.norm(Xm - Xr, axis=1) / np.linalg.norm(Xr, axis=1))),
               "rcs_db_err_max": float(np.max(np.abs(10 * np.log10(rcs / rcs_r))))}
    return dict(N=N, R=R, total=total, total_unprofiled=total_unprofiled, setup=np.array(setup_t),
                solve=np.array(solve_t), rcs=rcs,
                ratio=ratio, stats=stats, err=err)


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
        h = hps.hps_create(0, stream)
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

    def batch_ctx(precision):
        c = hps.hps_batch_create(P, 0, stream)
        for p, (xyz, tri) in enumerate(bw["meshes"]):
            hps.hps_batch_set_mesh(c, p, xyz, tri)
        prm.precision, prm.refine_passes = precision, (1 if precision else 0)
        for p, a in enumerate(parts):
            hps.hps_batch_set_hmatrix(c, p, prm, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"],
                                      a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        prm.precision, prm.refine_passes = 0, 0
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

    def run_batch(c, precision):
        Xb = torch.zeros(R * NT, dtype=torch.complex128, device="cuda")
        timed(c, Xb, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        su, so, rcs, ratio = timed(c, Xb, args.steps)
        torch.cuda.synchronize()
        return dict(total=time.perf_counter() - t0, setup=su, solve=so, rcs=rcs, X=Xb.cpu().numpy())

    ctx = batch_ctx(0)
    res = {0: run_batch(ctx, 0)}
    st = hps.hps_stats(ctx)
    hps.hps_destroy(ctx)
    print("[bench] batched FP64 done", file=sys.stderr, flush=True)
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
        c = hps.hps_create(0, stream)
        hps.hps_set_mesh(c, xyz, tri)
        a = parts[p]
        hps.hps_set_hmatrix(c, prm, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"], a["near_vals"],
                            a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        Xp = torch.zeros((R, Ns[p]), dtype=torch.complex128, device="cuda")
        timed(c, Xp, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        su, so, rcs_p, _ = timed(c, Xp, args.steps)
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
        res[2]["err"] = max(res[2].get("err", 0.0),
                            float(np.max(np.linalg.norm(xb - x4, axis=1) / np.linalg.norm(x4, axis=1))))
        worst_db = max(worst_db, float(np.max(np.abs(10 * np.log10(res[2]["rcs"][p] / rcs4)))))
        off += Ns[p]
        hps.hps_destroy(c)
        print("[bench] plain problem %d/%d done" % (p + 1, P), file=sys.stderr, flush=True)
    K = args.steps
    out = {"workload": bw["name"], "problems": P, "rhs_per_problem": R, "unknowns": NT,
           "unknowns_min_max": [min(Ns), max(Ns)], "hmatrix_build_s": build_s,
           "plain_sequential": {"rhs_per_s_step": P * R * K / seq_total, "setup_s": seq_setup,
                                "solve_rhs_per_s": P * R / seq_solve}}
    for form, name in ((0, "batched_fp64"), (2, "batched_mixed_fp16_far")):
        r = res[form]
        out[name] = {"rhs_per_s_step": P * R * K / r["total"], "setup_s": float(np.median(r["setup"])),
                     "solve_rhs_per_s": P * R / float(np.median(r["solve"])),
                     "speedup_step_vs_plain": (P * R * K / r["total"]) / (P * R * K / seq_total)}
    out["batched_fp64"]["current_rel_err_vs_plain"] = worst
    out["batched_mixed_fp16_far"]["current_rel_err_vs_fp64_terms4"] = res[2].get("err")
    out["batched_mixed_fp16_far"]["rcs_db_err_vs_fp64_terms4"] = worst_db
    out["device_stats_fp16_form"] = {k: dev.get(k) for k in ("levels", "upper_blocks", "factor_bytes", "times_ms")}
    out["hmatrix"] = st.get("hmatrix")
    return out


def cpu_leg(args, w):
    """The oracle, untuned, on the host cores: its own H-matrix (untimed),
    its setup (timed) and the solve of the first --cpu-rhs RHS (timed)."""
    from threadpoolctl import threadpool_info
    from oracle.hmatrix import build_hmatrix
    from oracle.planewave import excitation
    from oracle.scaling import group_graph, min_degree_order, schur_scaling
    from oracle.series import PowerSeries
    workers = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    H = build_hmatrix(w["xyz"], w["tri"], w["freq_hz"], w["leaf_max"], w["aca_tol"], workers=workers,
                      open_surface=w.get("open", False))
    print("[bench] oracle H-matrix built in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    S = schur_scaling(H, min_degree_order(group_graph(H)))
    setup_s = time.perf_counter() - t0
    print("[bench] oracle setup %.1f s" % setup_s, file=sys.stderr, flush=True)
    R = args.cpu_rhs
    b = excitation(H.rwg, w["freq_hz"], w["khat"][:R], w["pol"][:R])
    t0 = time.perf_counter()
    PowerSeries(H, S).solve_rwg(b, 2)
    solve_s = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": R / solve_s, "unit": "RHS/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of the %d RHS (theta = 0..%d deg) of the same workload, two-term solve "
                      "after the oracle's own H-matrix build (%d worker processes, untimed) and setup"
                      % (R, len(w["khat"]), R - 1, workers),
            "setup_s": setup_s, "host_cpus": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    from workloads import workload
    w = workload(args.workload)
    hm, build_s = build_hmatrix(w)
    print("[bench] workload %s: %d unknowns, %d RHS" % (args.workload, hm["N"], len(w["khat"])), file=sys.stderr,
          flush=True)
    g = gpu_leg(args, w, hm)
    mixed = None
    if not args.no_mixed:
        forms = {}

        def form(gm, **more):
            return dict({"rhs_per_s_step": gm["R"] * args.steps / gm["total"],
                         "rhs_per_s_step_unprofiled": gm["R"] * args.steps / gm["total_unprofiled"],
                         "setup_s": float(np.median(gm["setup"])),
                         "solve_rhs_per_s": float(gm["R"] / np.median(gm["solve"])),
                         "speedup_solve_vs_plain_fp64": float(np.median(g["solve"]) / np.median(gm["solve"])),
                         "speedup_step_unprofiled_vs_plain_fp64": float(g["total_unprofiled"] /
                                                                        gm["total_unprofiled"]),
                         "accuracy_vs_fp64": gm["err"]}, **more)

        for prec, name in ((1, "bf16_far"), (2, "fp16_far")):
            forms[name] = form(gpu_leg(args, w, hm, precision=prec, refine=1, reference_terms=4), residual_passes=1)
        # the same FP32 / FP16 operands without the residual pass: the
        # two-term series itself, against the FP64 two-term series
        forms["fp16_far_two_terms"] = form(gpu_leg(args, w, hm, precision=2, refine=0, reference_terms=2),
                                           residual_passes=0)
        mixed = {"form": "FP32 near operands on MFMA, 16-bit far factors with per-block FP32 scale, "
                         "FP64 setup; bf16_far / fp16_far add one FP32 residual pass (= four-term series)",
                 "variants": forms}
    cfie = None
    if not args.no_cfie and not w.get("open"):
        # CFIE of eq. (8), alpha = 0.5, on the same mesh: its own H-matrix
        # (both orders of every block), left and right coefficients; accuracy
        # of the two-term series against the converged series
        extra = {"formulation": 1, "cfie_alpha": 0.5}
        hc, bc = build_hmatrix(w, **extra)
        gc = gpu_leg(args, w, hc, extra=extra, reference_terms=60, reference_tol=1e-10)
        dc = gc["stats"].get("device", {})
        cfie = {"form": "CFIE alpha 0.5, plain fp64, two terms",
                "rhs_per_s_step": gc["R"] * args.steps / gc["total"],
                "ms_per_step": 1e3 * gc["total"] / args.steps,
                "setup_s": float(np.median(gc["setup"])),
                "solve_rhs_per_s": float(gc["R"] / np.median(gc["solve"])),
                "hmatrix_build_s": bc, "ratio_max": float(np.max(gc["ratio"])),
                "ratio_median": float(np.median(gc["ratio"])),
                "two_terms_vs_converged_series": gc["err"],
                "factor_bytes": dc.get("factor_bytes"), "upper_blocks": dc.get("upper_blocks")}
        # the series run until ||it_t|| / ||it_0|| < 1e-4 for every RHS (eq. 45
        # ratio control), against the same converged reference
        ea = dict(extra, terms=40, series_tol=1e-4)
        ga = gpu_leg(args, w, hc, extra=ea, reference_terms=60, reference_tol=1e-10)
        cfie["adaptive_series_1e-4"] = {
            "rhs_per_s_step": ga["R"] * args.steps / ga["total"],
            "solve_rhs_per_s": float(ga["R"] / np.median(ga["solve"])),
            "terms_used": ga["stats"].get("device", {}).get("terms_used"),
            "vs_converged_series": ga["err"]}
    R, K = g["R"], args.steps
    ms_per_step = 1e3 * g["total"] / K
    dev = dict(g["stats"].get("device", {}))
    log = dev.pop("launch_log", None) or []
    k = dev.get("kernels", {}).get(DOMINANT, {})
    # the dominant kernel's launches by size (algorithmic bytes per launch):
    # large ones stream, small ones (chain levels, few tiles) are latency-bound
    classes = []
    sub = [x for x in log if x[0] == 1 and len(x) >= 5]
    for lo, hi in ((0, 1e7), (1e7, 1e8), (1e8, 1e9), (1e9, float("inf"))):
        sel = [x for x in sub if lo <= x[3] < hi]
        if sel:
            b, f, t = sum(x[3] for x in sel), sum(x[2] for x in sel), sum(x[4] for x in sel) * 1e-3
            classes.append({"bytes_per_launch": [lo, hi if hi != float("inf") else None],
                            "launches_per_step": len(sel) / args.steps, "ms_per_step": 1e3 * t / args.steps,
                            "achieved_gb_s": b / t / 1e9, "hbm_frac": b / t / PEAK["hbm"],
                            "achieved_tflops": f / t / 1e12, "intensity_flop_per_byte": f / b})
    roofline = None
    if k.get("ms") and k.get("bytes"):
        sec = k["ms"] * 1e-3
        flop_rate, byte_rate = k["flops"] / sec, k["bytes"] / sec
        # roofline of the kernel: its algorithmic intensity (flops per
        # algorithmic byte) against the ridge point of FP64 MFMA over HBM
        intensity = k["flops"] / k["bytes"]
        ridge = PEAK["fp64"] / PEAK["hbm"]
        if intensity < ridge:
            bound, achieved, peak, unit = "hbm", byte_rate / 1e9, PEAK["hbm"] / 1e9, "GB/s"
        else:
            bound, achieved, peak, unit = "mfma", flop_rate / 1e12, PEAK["fp64"] / 1e12, "TFLOP/s"
        roofline = {"kernel": "k_gemm<1> (grouped complex GEMM on FP64 MFMA, subtract)", "bound": bound,
                    "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                    "traffic": counted_traffic(args.workload),
                    "algorithmic_bytes_per_launch": k["bytes"] / k["launches"],
                    "flops_per_launch": k["flops"] / k["launches"],
                    "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                    "attainable_tflops": min(PEAK["fp64"], intensity * PEAK["hbm"]) / 1e12,
                    "achieved_tflops": flop_rate / 1e12, "frac_of_fp64_mfma_peak": flop_rate / PEAK["fp64"],
                    "launches_per_step": k["launches"] / K, "avg_launch_us": 1e3 * k["ms"] / k["launches"],
                    "by_launch_size": classes}
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": g["N"], "rhs": R, "leaf_max": w["leaf_max"],
                   "aca_tol": w["aca_tol"], "freq_hz": w["freq_hz"], "form": "plain fp64", "terms": 2},
        "setup_s": float(np.median(g["setup"])),
        "solve_rhs_per_s": float(R / np.median(g["solve"])),
        "unprofiled": {"ms_per_step": 1e3 * g["total_unprofiled"] / K,
                       "rhs_per_s": R * K / g["total_unprofiled"],
                       "note": "the same K steps after the timed ones, without the per-launch HIP events "
                               "(solves replayed from their captured graph)"},
        "hmatrix_build_s": build_s,
        "ratio_max": float(np.max(g["ratio"])),
        "roofline": roofline,
        "precision_form": mixed,
        "cfie_form": cfie,
        "batching_form": batch_leg(args) if args.batch else None,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_leg(args, w),
        "device_stats": dev,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
