"""hps_hmatvec_noalloc (the allocation-free H-matrix product, whose work
vectors live in a fixed device scratch array) against hps_hmatvec on the same
context: two calls in a row, the second with fewer columns, so the second
reads a scratch array that still holds the first call's (larger) contents.
Both run the same kernels in the same order, so the products are bitwise
equal (FP64, and the FP32 precision form).  Also: host memory and a column
count beyond the scratch limit are refused before any launch.

The oracle's H-matrix of the 480-unknown sphere (icosphere subdivision 2,
300 MHz, leaf <= 16) is installed in the library, and the FP64 product is
also held against the oracle's H x to 1e-12.
"""

import numpy as np
import pytest

from oracle.hmatrix import build_hmatrix
from workloads import icosphere
from hmat_io import hmatrix_arrays

torch = pytest.importorskip("torch")
from paper_2109_04129_amd import hps  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sphere():
    xyz, tri = icosphere(2, 1.0)
    H = build_hmatrix(xyz, tri, 300e6, 16, 1e-3, workers=8)
    return xyz, tri, H


def _ctx(xyz, tri, H, precision):
    ctx = hps.hps_create(0, torch.cuda.current_stream().cuda_stream)
    hps.hps_set_mesh(ctx, xyz, tri)
    p = hps.hps_params_default(freq_hz=300e6, leaf_max=16, aca_tol=1e-3, terms=2, precision=precision,
                               refine_passes=1 if precision else 0)
    a = hmatrix_arrays(H)
    hps.hps_set_hmatrix(ctx, p, a["N"], a["perm"], a["group_ptr"], a["near_ts"], a["near_off"], a["near_vals"],
                        a["far_rng"], a["far_rank"], a["far_off"], a["far_uv"])
    hps.hps_setup(ctx)
    return ctx


def _rand(N, R, seed):
    g = torch.Generator().manual_seed(seed)
    x = torch.randn((R, N), dtype=torch.complex128, generator=g)
    return x.to("cuda")


@pytest.mark.parametrize("precision", [0, 2])
def test_noalloc_matches_hmatvec(sphere, precision):
    xyz, tri, H = sphere
    N = H.N
    print("case: hmatvec_noalloc, 480 unknowns, precision %d, R = 37 then 5" % precision, flush=True)
    ctx = _ctx(xyz, tri, H, precision)
    try:
        for R, seed in ((37, 1), (5, 2)):
            X = _rand(N, R, seed)
            Y0 = torch.zeros_like(X)
            Y1 = torch.full_like(X, complex(np.nan, np.nan))
            hps.hps_hmatvec(ctx, R, X.data_ptr(), Y0.data_ptr())
            hps.hps_hmatvec_noalloc(ctx, R, X.data_ptr(), Y1.data_ptr())
            torch.cuda.synchronize()
            y0, y1 = Y0.cpu().numpy(), Y1.cpu().numpy()
            assert np.array_equal(y0, y1), "R=%d: max |diff| %.3e" % (R, np.max(np.abs(y0 - y1)))
            if precision == 0:
                xh = X.cpu().numpy().T
                ref = H.to_rwg(H.matvec(H.to_tree(xh))).T
                err = np.linalg.norm(y1 - ref) / np.linalg.norm(ref)
                print("R=%d: bitwise equal to hps_hmatvec; vs oracle H x %.2e" % (R, err), flush=True)
                assert err < 1e-12
    finally:
        hps.hps_destroy(ctx)


def test_noalloc_refuses_host_memory_and_oversize(sphere):
    xyz, tri, H = sphere
    N = H.N
    ctx = _ctx(xyz, tri, H, 0)
    try:
        Xh = np.zeros((2, N), dtype=np.complex128)
        Y = torch.zeros((2, N), dtype=torch.complex128, device="cuda")
        with pytest.raises(hps.HpsError) as e:
            hps.hps_hmatvec_noalloc(ctx, 2, Xh.ctypes.data, Y.data_ptr())
        assert e.value.status == -1
        t_rows = hps.hps_stats(ctx)["device"]["far_T_rows"]
        per_col = 16 * (2 * N + t_rows)
        R = (64 << 20) // per_col + 8          # beyond the 64 MiB scratch: refused before any launch
        X = torch.zeros((R, N), dtype=torch.complex128, device="cuda")
        Y = torch.zeros_like(X)
        with pytest.raises(hps.HpsError) as e:
            hps.hps_hmatvec_noalloc(ctx, R, X.data_ptr(), Y.data_ptr())
        assert e.value.status == -1
        assert "scratch" in str(e.value)
        print("refused R=%d: %s" % (R, e.value), flush=True)
    finally:
        hps.hps_destroy(ctx)
