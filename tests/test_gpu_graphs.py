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
