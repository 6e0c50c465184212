"""ctypes binding of include/hps.h (argument marshalling only).

Device arrays are passed as raw pointers (e.g. ``tensor.data_ptr()`` of a
complex128 CUDA/HIP tensor); host arrays as NumPy arrays.  Every function
raises ``HpsError`` on a negative status; HPS_WRATIO (1) is returned as is.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhps.so")

HPS_OK, HPS_WRATIO = 0, 1
STATUS = {0: "HPS_OK", 1: "HPS_WRATIO", -1: "HPS_EINVAL", -2: "HPS_ENOMEM", -3: "HPS_EDEVICE",
          -4: "HPS_ESINGULAR", -5: "HPS_ESTATE", -6: "HPS_EIO"}

EXPORTS = ["hps_params_default", "hps_create", "hps_destroy", "hps_last_error", "hps_set_mesh",
           "hps_num_unknowns", "hps_build_hmatrix", "hps_set_hmatrix", "hps_hmatrix_sizes",
           "hps_get_hmatrix", "hps_setup", "hps_solve_planewaves", "hps_solve_rhs",
           "hps_excitation", "hps_hmatvec", "hps_hmatvec_noalloc", "hps_set_tuning", "hps_profile", "hps_stats", "hps_batch_create",
           "hps_batch_set_mesh", "hps_batch_set_hmatrix", "hps_num_problems", "hps_problem_unknowns",
           "hps_set_open_mesh", "hps_rwg", "hps_export_hmatrix", "hps_import_hmatrix"]


class HpsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class hps_params(ctypes.Structure):
    _fields_ = [("freq_hz", ctypes.c_double), ("leaf_max", ctypes.c_int32),
                ("aca_tol", ctypes.c_double), ("precision", ctypes.c_int32),
                ("terms", ctypes.c_int32), ("refine_passes", ctypes.c_int32),
                ("ratio_warn", ctypes.c_double), ("device_mem_cap", ctypes.c_uint64),
                ("host_threads", ctypes.c_int32), ("ordering", ctypes.c_int32),
                ("graphs", ctypes.c_int32), ("verbose", ctypes.c_int32),
                ("leaf_box_min", ctypes.c_double), ("series_tol", ctypes.c_double),
                ("host_near", ctypes.c_int32), ("formulation", ctypes.c_int32),
                ("cfie_alpha", ctypes.c_double), ("eta", ctypes.c_double)]


_lib = None


def lib():
    """Load libhps.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime (same soname as the system one).
        # Importing it first makes libhps bind to that copy, so device
        # pointers and streams from torch are valid in the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhps.so is not built; run python -m paper_2109_04129_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32, d, vp = ctypes.POINTER, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
        ctx = vp
        L.hps_params_default.argtypes = [P(hps_params)]
        L.hps_create.argtypes = [P(ctx), ctypes.c_int, vp]
        L.hps_destroy.argtypes = [ctx]
        L.hps_destroy.restype = None
        L.hps_last_error.argtypes = [ctx]
        L.hps_last_error.restype = ctypes.c_char_p
        L.hps_set_mesh.argtypes = [ctx, vp, i64, vp, i64]
        L.hps_set_open_mesh.argtypes = [ctx, vp, i64, vp, i64]
        L.hps_num_unknowns.argtypes = [ctx, P(i64)]
        L.hps_build_hmatrix.argtypes = [ctx, P(hps_params)]
        L.hps_set_hmatrix.argtypes = [ctx, P(hps_params), i64, vp, i64, vp, i64, vp, vp, vp,
                                      i64, vp, vp, vp, vp]
        L.hps_hmatrix_sizes.argtypes = [ctx, P(i64), P(i64), P(i64), P(i64), P(i64)]
        L.hps_get_hmatrix.argtypes = [ctx] + [vp] * 9
        L.hps_setup.argtypes = [ctx]
        L.hps_solve_planewaves.argtypes = [ctx, i64, vp, vp, vp, vp, vp]
        L.hps_solve_rhs.argtypes = [ctx, i64, vp, vp, vp]
        L.hps_excitation.argtypes = [ctx, i64, vp, vp, vp]
        L.hps_hmatvec.argtypes = [ctx, i64, vp, vp]
        L.hps_hmatvec_noalloc.argtypes = [ctx, i64, vp, vp]
        L.hps_set_tuning.argtypes = [ctx, ctypes.c_char_p]
        L.hps_stats.argtypes = [ctx, ctypes.c_char_p, ctypes.c_size_t]
        L.hps_profile.argtypes = [ctx, ctypes.c_int]
        L.hps_batch_create.argtypes = [P(ctx), ctypes.c_int, vp, i32]
        L.hps_batch_set_mesh.argtypes = [ctx, i32, vp, i64, vp, i64]
        L.hps_batch_set_hmatrix.argtypes = [ctx, i32, P(hps_params), i64, vp, i64, vp, i64, vp, vp, vp,
                                            i64, vp, vp, vp, vp]
        L.hps_num_problems.argtypes = [ctx, P(i32)]
        L.hps_problem_unknowns.argtypes = [ctx, i32, P(i64)]
        L.hps_rwg.argtypes = [ctx, vp, vp, vp]
        L.hps_export_hmatrix.argtypes = [ctx, ctypes.c_char_p]
        L.hps_import_hmatrix.argtypes = [ctx, ctypes.c_char_p]
        for name in EXPORTS:
            if name not in ("hps_destroy", "hps_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(ctx, st):
    if st < 0:
        msg = lib().hps_last_error(ctx).decode() if ctx else ""
        raise HpsError(st, msg)
    return st


def hps_params_default(**kw):
    p = hps_params()
    lib().hps_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def hps_create(device=0, stream=None):
    c = ctypes.c_void_p()
    st = lib().hps_create(ctypes.byref(c), int(device), stream)
    if st < 0:
        raise HpsError(st, "hps_create failed: " + lib().hps_last_error(None).decode())
    return c


def hps_destroy(ctx):
    lib().hps_destroy(ctx)


def hps_last_error(ctx):
    return lib().hps_last_error(ctx).decode()


def hps_set_mesh(ctx, xyz, tri):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    return _check(ctx, lib().hps_set_mesh(ctx, _ptr(xyz), len(xyz), _ptr(tri), len(tri)))


def hps_set_open_mesh(ctx, xyz, tri):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    return _check(ctx, lib().hps_set_open_mesh(ctx, _ptr(xyz), len(xyz), _ptr(tri), len(tri)))


def hps_num_unknowns(ctx):
    n = ctypes.c_int64()
    _check(ctx, lib().hps_num_unknowns(ctx, ctypes.byref(n)))
    return n.value


def hps_build_hmatrix(ctx, params):
    return _check(ctx, lib().hps_build_hmatrix(ctx, ctypes.byref(params)))


def _hmatrix_args(N, perm, group_ptr, near_ts, near_off, near_vals, far_rng, far_rank, far_off, far_uv):
    perm = np.ascontiguousarray(perm, dtype=np.int64)
    group_ptr = np.ascontiguousarray(group_ptr, dtype=np.int64)
    near_ts = np.ascontiguousarray(near_ts, dtype=np.int32)
    near_off = np.ascontiguousarray(near_off, dtype=np.int64)
    near_vals = np.ascontiguousarray(near_vals, dtype=np.complex128)
    far_rng = np.ascontiguousarray(far_rng, dtype=np.int64)
    far_rank = np.ascontiguousarray(far_rank, dtype=np.int32)
    far_off = np.ascontiguousarray(far_off, dtype=np.int64)
    far_uv = np.ascontiguousarray(far_uv, dtype=np.complex128)
    keep = (perm, group_ptr, near_ts, near_off, near_vals, far_rng, far_rank, far_off, far_uv)
    args = (int(N), _ptr(perm), len(group_ptr) - 1, _ptr(group_ptr), len(near_ts) // 2, _ptr(near_ts),
            _ptr(near_off), _ptr(near_vals), len(far_rank), _ptr(far_rng), _ptr(far_rank), _ptr(far_off),
            _ptr(far_uv))
    return keep, args


def hps_set_hmatrix(ctx, params, N, perm, group_ptr, near_ts, near_off, near_vals,
                    far_rng, far_rank, far_off, far_uv):
    keep, args = _hmatrix_args(N, perm, group_ptr, near_ts, near_off, near_vals, far_rng, far_rank, far_off,
                               far_uv)
    return _check(ctx, lib().hps_set_hmatrix(ctx, ctypes.byref(params), *args))


def hps_batch_create(n_problems, device=0, stream=None):
    c = ctypes.c_void_p()
    st = lib().hps_batch_create(ctypes.byref(c), int(device), stream, int(n_problems))
    if st < 0:
        raise HpsError(st, "hps_batch_create failed: " + lib().hps_last_error(None).decode())
    return c


def hps_batch_set_mesh(ctx, p, xyz, tri):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    return _check(ctx, lib().hps_batch_set_mesh(ctx, int(p), _ptr(xyz), len(xyz), _ptr(tri), len(tri)))


def hps_batch_set_hmatrix(ctx, p, params, N, perm, group_ptr, near_ts, near_off, near_vals,
                          far_rng, far_rank, far_off, far_uv):
    keep, args = _hmatrix_args(N, perm, group_ptr, near_ts, near_off, near_vals, far_rng, far_rank, far_off,
                               far_uv)
    return _check(ctx, lib().hps_batch_set_hmatrix(ctx, int(p), ctypes.byref(params), *args))


def hps_num_problems(ctx):
    n = ctypes.c_int32()
    _check(ctx, lib().hps_num_problems(ctx, ctypes.byref(n)))
    return n.value


def hps_problem_unknowns(ctx, p):
    n = ctypes.c_int64()
    _check(ctx, lib().hps_problem_unknowns(ctx, int(p), ctypes.byref(n)))
    return n.value


def hps_hmatrix_sizes(ctx):
    v = [ctypes.c_int64() for _ in range(5)]
    _check(ctx, lib().hps_hmatrix_sizes(ctx, *[ctypes.byref(x) for x in v]))
    return dict(zip(["M", "n_near", "n_far", "near_elems", "far_elems"], [x.value for x in v]))


def hps_get_hmatrix(ctx):
    s = hps_hmatrix_sizes(ctx)
    N = hps_num_unknowns(ctx)
    out = dict(perm=np.empty(N, np.int64), group_ptr=np.empty(s["M"] + 1, np.int64),
               near_ts=np.empty(2 * s["n_near"], np.int32), near_off=np.empty(s["n_near"] + 1, np.int64),
               near_vals=np.empty(s["near_elems"], np.complex128),
               far_rng=np.empty(4 * s["n_far"], np.int64), far_rank=np.empty(s["n_far"], np.int32),
               far_off=np.empty(s["n_far"] + 1, np.int64), far_uv=np.empty(s["far_elems"], np.complex128))
    _check(ctx, lib().hps_get_hmatrix(ctx, *[_ptr(out[k]) for k in (
        "perm", "group_ptr", "near_ts", "near_off", "near_vals", "far_rng", "far_rank", "far_off", "far_uv")]))
    return out


def hps_rwg(ctx):
    """(edge_v, tri_pm, free_v), each N x 2 int32, RWG order."""
    N = hps_num_unknowns(ctx)
    out = [np.empty((N, 2), np.int32) for _ in range(3)]
    _check(ctx, lib().hps_rwg(ctx, *[_ptr(a) for a in out]))
    return tuple(out)


def hps_export_hmatrix(ctx, path):
    return _check(ctx, lib().hps_export_hmatrix(ctx, os.fsencode(path)))


def hps_import_hmatrix(ctx, path):
    return _check(ctx, lib().hps_import_hmatrix(ctx, os.fsencode(path)))


def hps_setup(ctx):
    return _check(ctx, lib().hps_setup(ctx))


def hps_solve_planewaves(ctx, khat, pol, X_ptr=None, want_rcs=True, want_ratio=True):
    khat = np.ascontiguousarray(khat, dtype=np.float64).reshape(-1, 3)
    pol = np.ascontiguousarray(pol, dtype=np.float64).reshape(-1, 3)
    R = len(khat)
    P = hps_num_problems(ctx)
    rcs = np.empty(P * R) if want_rcs else None
    ratio = np.empty(P * R) if want_ratio else None
    st = _check(ctx, lib().hps_solve_planewaves(ctx, R, _ptr(khat), _ptr(pol),
                                                ctypes.c_void_p(X_ptr) if X_ptr else None,
                                                _ptr(rcs), _ptr(ratio)))
    if P > 1:       # batch: (P, R), problem-major
        rcs = None if rcs is None else rcs.reshape(P, R)
        ratio = None if ratio is None else ratio.reshape(P, R)
    return st, rcs, ratio


def hps_solve_rhs(ctx, R, B_ptr, X_ptr, want_ratio=True):
    P = hps_num_problems(ctx)
    ratio = np.empty(P * R) if want_ratio else None
    st = _check(ctx, lib().hps_solve_rhs(ctx, int(R), ctypes.c_void_p(B_ptr), ctypes.c_void_p(X_ptr),
                                         _ptr(ratio)))
    if P > 1 and ratio is not None:
        ratio = ratio.reshape(P, R)
    return st, ratio


def hps_excitation(ctx, khat, pol, B_ptr):
    khat = np.ascontiguousarray(khat, dtype=np.float64).reshape(-1, 3)
    pol = np.ascontiguousarray(pol, dtype=np.float64).reshape(-1, 3)
    return _check(ctx, lib().hps_excitation(ctx, len(khat), _ptr(khat), _ptr(pol), ctypes.c_void_p(B_ptr)))


def hps_hmatvec(ctx, R, X_ptr, Y_ptr):
    return _check(ctx, lib().hps_hmatvec(ctx, int(R), ctypes.c_void_p(X_ptr), ctypes.c_void_p(Y_ptr)))


def hps_hmatvec_noalloc(ctx, R, X_ptr, Y_ptr):
    return _check(ctx, lib().hps_hmatvec_noalloc(ctx, int(R), ctypes.c_void_p(X_ptr), ctypes.c_void_p(Y_ptr)))


def hps_set_tuning(ctx, path):
    return _check(ctx, lib().hps_set_tuning(ctx, None if path is None else str(path).encode()))


def hps_profile(ctx, enable=True):
    return _check(ctx, lib().hps_profile(ctx, 1 if enable else 0))


def hps_stats(ctx):
    import json
    buf = ctypes.create_string_buffer(1 << 24)
    _check(ctx, lib().hps_stats(ctx, buf, len(buf)))
    return json.loads(buf.value.decode())
