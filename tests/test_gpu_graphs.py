"""Graph replay of the solve against eager launches.

The device part of hps_solve_planewaves / hps_solve_rhs is captured once per
RHS count and replayed.  Every replay, with other device work and host
synchronisations in between and with changes of the RHS count (re-capture),
must reproduce the eager launches bit for bit (same kernels, same order)."""

import numpy as np
import pytest

from hmat_io import hmatrix_arrays
from workloads import monostatic_angles

torch = pytest.importorskip("torch")
from paper_2109_04129_amd import hps  # noqa: E402

pytestmark = pytest.mark.gpu


def _ctx(H, xyz, tri, graphs, precision):
    ctx = hps.hps_create(0, torch.cuda.current_stream().cuda_stream)
    hps.hps_set_mesh(ctx, xyz, tri)
    p = hps.hps_params_default(freq_hz=300e6, leaf_max=16, aca_tol=1e-3, terms=2, graphs=graphs,
                               precision=precision, refine_passes=1 if precision else 0)
    a = hmatrix_arrays(H)
    hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"], a["near_vals"],
                        a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
    hps.hps_setup(ctx)
    return ctx


@pytest.mark.parametrize("precision", [0, 2])
def test_graph_replays_match_eager(small_sphere, precision):
    from workloads import icosphere
    xyz, tri = icosphere(2, 1.0)
    H = small_sphere
    N = H.N
    print("case: graph replays vs eager, 480 unknowns, precision", precision, flush=True)
    eager = _ctx(H, xyz, tri, 0, precision)
    graph = _ctx(H, xyz, tri, 1, precision)
    try:
        rng = np.random.default_rng(3)
        for R in (5, 3, 5, 1):
            th = rng.uniform(0, 180, R)
            ph = rng.uniform(0, 360, R)
            khat, pol = monostatic_angles(th, ph)
            Xe = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
            _, rcs_e, rat_e = hps.hps_solve_planewaves(eager, khat, pol, Xe.data_ptr())
            B = torch.randn((R, N), dtype=torch.complex128, device="cuda")
            Ye = torch.zeros_like(B)
            _, rb_e = hps.hps_solve_rhs(eager, R, B.data_ptr(), Ye.data_ptr())
            torch.cuda.synchronize()
            for rep in range(3):
                junk = torch.randn(1 << 16, dtype=torch.float64, device="cuda")     # other device work
                junk = (junk * 2.0).sum()
                torch.cuda.synchronize()
                Xg = torch.zeros_like(Xe)
                _, rcs_g, rat_g = hps.hps_solve_planewaves(graph, khat, pol, Xg.data_ptr())
                Yg = torch.zeros_like(B)
                _, rb_g = hps.hps_solve_rhs(graph, R, B.data_ptr(), Yg.data_ptr())
                torch.cuda.synchronize()
                assert torch.equal(Xg, Xe), (R, rep)
                assert torch.equal(Yg, Ye), (R, rep)
                assert np.array_equal(rcs_g, rcs_e) and np.array_equal(rat_g, rat_e)
                assert np.array_equal(rb_g, rb_e)
    finally:
        hps.hps_destroy(eager)
        hps.hps_destroy(graph)


def _set(ctx, p, a):
    hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"], a["near_vals"],
                        a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])


def _perturbed(a, seed):
    """The same H-matrix structure with other values: every near entry and
    far factor entry scaled by a random complex factor near 1."""
    rng = np.random.default_rng(seed)
    b = dict(a)
    for key in ("near_vals", "far_uv"):
        v = np.asarray(a[key])
        f = 1.0 + 0.05 * (rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape))
        b[key] = v * f
    return b


def _solve_both(ctx, N, khat, pol, B):
    R = len(khat)
    X = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
    _, rcs, rat = hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
    Y = torch.zeros_like(B)
    _, rb = hps.hps_solve_rhs(ctx, R, B.data_ptr(), Y.data_ptr())
    torch.cuda.synchronize()
    return X.cpu().numpy(), Y.cpu().numpy(), rcs, rat, rb


@pytest.mark.parametrize("precision", [0, 2])
def test_setup_replays_match_eager(small_sphere, precision):
    """graphs = 2: setups of an unchanged structure replay the recorded
    launches from a captured graph on the values installed since (other
    values, same structure), with other device work and synchronisations in
    between; every replay matches an eager context holding the same values
    bit for bit, and a new structure falls back to an eager setup."""
    from workloads import icosphere
    from oracle.hmatrix import build_hmatrix
    xyz, tri = icosphere(2, 1.0)
    H = small_sphere
    N = H.N
    print("case: setup replays vs eager setups, 480 unknowns, precision", precision, flush=True)
    a0 = hmatrix_arrays(H)
    a1 = _perturbed(a0, 11)
    H2 = build_hmatrix(xyz, tri, 300e6, 8, 1e-3, workers=8)       # another structure (leaves of 8: 176 groups)
    a2 = hmatrix_arrays(H2)
    p = hps.hps_params_default(freq_hz=300e6, leaf_max=16, aca_tol=1e-3, terms=2, graphs=2,
                               precision=precision, refine_passes=1 if precision else 0)
    pe = hps.hps_params_default(freq_hz=300e6, leaf_max=16, aca_tol=1e-3, terms=2, graphs=0,
                                precision=precision, refine_passes=1 if precision else 0)
    khat, pol = monostatic_angles([0.0, 45.0, 90.0, 180.0, 33.0], [0.0, 10.0, 200.0, 0.0, 77.0])
    g = torch.Generator().manual_seed(5)
    B = torch.complex(torch.randn((5, N), generator=g, dtype=torch.float64),
                      torch.randn((5, N), generator=g, dtype=torch.float64)).cuda()
    ref = {}
    for name, a in (("a0", a0), ("a1", a1), ("a2", a2)):
        e = hps.hps_create(0, torch.cuda.current_stream().cuda_stream)
        try:
            hps.hps_set_mesh(e, xyz, tri)
            _set(e, pe, a)
            hps.hps_setup(e)
            ref[name] = _solve_both(e, N, khat, pol, B)
        finally:
            hps.hps_destroy(e)
    ctx = hps.hps_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        hps.hps_set_mesh(ctx, xyz, tri)
        # (values installed before the setup or None: setup again as is, expected replay count)
        seq = [("a0", True, 0), ("a0", False, 1), ("a1", True, 2), ("a0", True, 3), ("a0", False, 4),
               ("a2", True, 4), ("a2", False, 5), ("a0", True, 5), ("a1", True, 6)]
        for step, (name, install, replays) in enumerate(seq):
            junk = torch.randn(1 << 16, dtype=torch.float64, device="cuda")     # other device work
            junk = (junk * 2.0).sum()
            torch.cuda.synchronize()
            if install:
                _set(ctx, p, {"a0": a0, "a1": a1, "a2": a2}[name])
            hps.hps_setup(ctx)
            got = _solve_both(ctx, N, khat, pol, B)
            st = hps.hps_stats(ctx)["device"]
            print("step", step, name, "replays", st["setup_replays"], flush=True)
            assert st["setup_replays"] == replays, (step, st["setup_replays"])
            for u, v in zip(got, ref[name]):
                assert np.array_equal(u, v), (step, name)
    finally:
        hps.hps_destroy(ctx)


def test_batch_setup_replays_match_eager():
    """The batching form with graphs = 2: three problems in one context,
    problem 1's values changed between setups; each replayed setup matches
    an eager batch context holding the same values bit for bit."""
    from oracle.hmatrix import build_hmatrix
    from workloads import ellipsoid_mesh, icosphere
    xyz1, tri1 = icosphere(1, 1.0)
    xyz2, tri2 = icosphere(2, 1.0)
    xyz3, tri3 = ellipsoid_mesh(xyz2, tri2, (1.3, 0.9, 0.6))
    meshes = [(xyz1, tri1), (xyz3, tri3), (0.8 * xyz2, tri2)]
    arrs = [hmatrix_arrays(build_hmatrix(x, t, 300e6, 16, 1e-3, workers=8)) for x, t in meshes]
    alt = _perturbed(arrs[1], 23)
    Ns = [a["N"] for a in arrs]
    khat, pol = monostatic_angles([0.0, 90.0, 180.0], [0.0, 45.0, 0.0])
    R = len(khat)
    print("case: batch of 3 (120/480/480 unknowns), setup replays vs eager", flush=True)

    def batch(graphs, variant):
        ctx = hps.hps_batch_create(3, 0, torch.cuda.current_stream().cuda_stream)
        p = hps.hps_params_default(freq_hz=300e6, leaf_max=16, aca_tol=1e-3, terms=2, graphs=graphs)
        for q, (x, t) in enumerate(meshes):
            hps.hps_batch_set_mesh(ctx, q, x, t)
        install(ctx, p, variant)
        return ctx, p

    def install(ctx, p, variant):
        for q, a in enumerate(arrs):
            a = alt if (q == 1 and variant == 1) else a
            hps.hps_batch_set_hmatrix(ctx, q, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"],
                                      a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])

    def solve(ctx):
        X = torch.zeros(R * sum(Ns), dtype=torch.complex128, device="cuda")
        _, rcs, rat = hps.hps_solve_planewaves(ctx, khat, pol, X.data_ptr())
        torch.cuda.synchronize()
        return X.cpu().numpy(), rcs, rat

    ref = []
    for variant in (0, 1):
        e, _ = batch(0, variant)
        try:
            hps.hps_setup(e)
            ref.append(solve(e))
        finally:
            hps.hps_destroy(e)
    ctx, p = batch(2, 0)
    try:
        for step, variant in enumerate([0, 0, 1, 0, 1, 1]):
            if step > 0 and variant != [0, 0, 1, 0, 1, 1][step - 1]:
                install(ctx, p, variant)
            hps.hps_setup(ctx)
            got = solve(ctx)
            assert hps.hps_stats(ctx)["device"]["setup_replays"] == step
            for u, v in zip(got, ref[variant]):
                assert np.array_equal(u, v), (step, variant)
    finally:
        hps.hps_destroy(ctx)
