"""Element-wise parity with the oracle at the full size of the 30,720-unknown
sphere (icosphere subdivision 5, 790 MHz, leaf <= 128, ACA 1e-3), in the
launch configuration bench.py times: all 181 monostatic RHS (theta = 0..180
deg) in one solve, so six RHS column tiles per target and the XCD-ordered
far-field and D^-1 launches.

The oracle builds its own H-matrix (its quadrature, tree and ACA) on host
worker processes, which is installed in the library, so both sides start
from the same Z_N and Z_F.  The oracle factors with its own minimum-degree
order and solves a sample of 8 RHS (theta = 0, 1, 45, 90, 133, 178, 179,
180 deg); the library sets up with its nested-dissection order.  Currents
and RCS do not depend on the order, so they are compared RHS by RHS:
currents to 1e-10 relative (FP64 rounding of two elimination orders), RCS to
1e-6 dB.  (The eq. (45) ratio lives in the scaled unknowns and depends on the
order; its parity is checked under a common order on the 1,920- and
480-unknown spheres, where the oracle can afford the natural order.)  The precision form (FP32 solve operands, 16-bit far factors, one
FP32 residual pass, i.e. the four-term series) is compared with the oracle's
four-term series at the 1e-3 current / 0.1 dB target.
"""

import os

import numpy as np
import pytest

from oracle.hmatrix import build_hmatrix
from oracle.planewave import excitation, monostatic_rcs
from oracle.scaling import group_graph, min_degree_order, schur_scaling
from oracle.series import PowerSeries
from workloads import workload
from hmat_io import hmatrix_arrays, per_rhs_rel

torch = pytest.importorskip("torch")
from paper_2109_04129_amd import hps  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

SAMPLE = [0, 1, 45, 90, 133, 178, 179, 180]


@pytest.fixture(scope="module")
def c1():
    w = workload("sphere_s5_790MHz")
    workers = min(16, os.cpu_count() or 1)
    print("case: sphere 30,720 unknowns, oracle H-matrix (%d workers), 181 RHS" % workers, flush=True)
    H = build_hmatrix(w["xyz"], w["tri"], w["freq_hz"], w["leaf_max"], w["aca_tol"], workers=workers)
    print("oracle H-matrix built: %d groups, %d far blocks" % (H.M, len(H.far)), flush=True)
    S = schur_scaling(H, min_degree_order(group_graph(H)))
    print("oracle setup done", flush=True)
    khat, pol = w["khat"][SAMPLE], w["pol"][SAMPLE]
    b = excitation(H.rwg, w["freq_hz"], khat, pol)
    ps = PowerSeries(H, S)
    x2, r2 = ps.solve_rwg(b, 2)
    x4, _ = ps.solve_rwg(b, 4)
    print("oracle solves done", flush=True)
    return dict(w=w, H=H, a=hmatrix_arrays(H), x2=x2, x4=x4, ratio2=r2[0],
                sig2=monostatic_rcs(H.rwg, w["freq_hz"], khat, pol, x2),
                sig4=monostatic_rcs(H.rwg, w["freq_hz"], khat, pol, x4))


def _run(c1, precision=0, refine=0):
    w, a = c1["w"], c1["a"]
    ctx = hps.hps_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        hps.hps_set_mesh(ctx, w["xyz"], w["tri"])
        p = hps.hps_params_default(freq_hz=w["freq_hz"], leaf_max=w["leaf_max"], aca_tol=w["aca_tol"], terms=2,
                                   precision=precision, refine_passes=refine)
        hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"],
                            a["near_vals"], a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
        hps.hps_setup(ctx)
        R = len(w["khat"])
        X = torch.zeros((R, a["N"]), dtype=torch.complex128, device="cuda")
        st, rcs, ratio = hps.hps_solve_planewaves(ctx, w["khat"], w["pol"], X.data_ptr())
        torch.cuda.synchronize()
        Xs = X[SAMPLE].cpu().numpy().T.copy()
    finally:
        hps.hps_destroy(ctx)
    return st, Xs, rcs[SAMPLE], ratio


def test_fp64_currents_and_rcs_elementwise(c1):
    st, X, rcs, ratio = _run(c1)
    err = per_rhs_rel(X, c1["x2"])
    db = np.abs(10 * np.log10(rcs / c1["sig2"]))
    print("FP64, 181 RHS: current rel err per sampled RHS", np.array2string(err, precision=2),
          "max RCS err %.2e dB" % db.max(), flush=True)
    assert err.max() < 1e-10
    assert db.max() < 1e-6
    assert st == (hps.HPS_WRATIO if np.any(ratio >= 0.1) else hps.HPS_OK)


@pytest.mark.parametrize("precision", [2, 1])
def test_precision_form_vs_four_term_oracle(c1, precision):
    st, X, rcs, ratio = _run(c1, precision=precision, refine=1)
    err = per_rhs_rel(X, c1["x4"])
    db = np.abs(10 * np.log10(rcs / c1["sig4"]))
    print("precision %d + 1 residual pass, 181 RHS: current rel err vs oracle four terms max %.3e, "
          "RCS max %.4f dB" % (precision, err.max(), db.max()), flush=True)
    assert err.max() < 1e-3
    assert db.max() < 0.1
