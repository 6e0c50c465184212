"""Marshal an oracle H-matrix into the flat arrays of hps_set_hmatrix and run
the library through the ctypes binding (test helper; no arithmetic of the
method lives here)."""

import numpy as np


def hmatrix_arrays(H):
    keys = sorted(H.near)
    near_ts = np.array(keys, dtype=np.int32).reshape(-1)
    sizes = [H.near[k].size for k in keys]
    near_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    near_vals = np.concatenate([H.near[k].reshape(-1) for k in keys])
    far_rng = np.array([(a, b, c, d) for a, b, c, d, _, _ in H.far], dtype=np.int64).reshape(-1)
    far_rank = np.array([U.shape[1] for *_, U, V in H.far], dtype=np.int32)
    parts = []
    for *_, U, V in H.far:
        parts.append(U.ravel(order="F"))
        parts.append(V.ravel(order="F"))
    fsz = [U.size + V.size for *_, U, V in H.far]
    far_off = np.concatenate([[0], np.cumsum(fsz)]).astype(np.int64)
    far_uv = np.concatenate(parts) if parts else np.zeros(0, np.complex128)
    group_ptr = np.concatenate([H.groups[:, 0], [H.N]]).astype(np.int64)
    return dict(N=H.N, perm=H.perm, group_ptr=group_ptr, near_ts=near_ts, near_off=near_off,
                near_vals=near_vals, far_rng=far_rng, far_rank=far_rank, far_off=far_off, far_uv=far_uv)


def per_rhs_rel(x, ref):
    return np.linalg.norm(x - ref, axis=0) / np.linalg.norm(ref, axis=0)


def dense_near_from_arrays(a):
    """Dense near field (tree order) of an H-matrix given as hps_set_hmatrix
    arrays; the (s, t) block is the transpose of the stored (t, s) one."""
    gp = a["group_ptr"]
    N = int(gp[-1])
    Z = np.zeros((N, N), dtype=np.complex128)
    for b, (t, s) in enumerate(np.asarray(a["near_ts"]).reshape(-1, 2)):
        m, n = gp[t + 1] - gp[t], gp[s + 1] - gp[s]
        B = a["near_vals"][a["near_off"][b]:a["near_off"][b + 1]].reshape(m, n)
        Z[gp[t]:gp[t + 1], gp[s]:gp[s + 1]] = B
        Z[gp[s]:gp[s + 1], gp[t]:gp[t + 1]] = B.T
    return Z
