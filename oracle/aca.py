"""Re-compressed adaptive cross approximation of an admissible block
(eqs. 11-12 and the re-compression of refs. [20, 21] cited in Sec. II).

ACA with partial pivoting builds Z_sub ~= sum_k u_k v_k^T from single rows and
columns of the block:

* the first pivot row is local row 0; row i_k of the residual is
  r = Z[i_k, :] - sum_l u_l[i_k] v_l; the pivot column j_k maximises |r_j|
  (lowest index on ties); v_k = r / r_{j_k};
* u_k = Z[:, j_k] - sum_l v_l[j_k] u_l (the residual column);
* ||S_k||_F^2 = ||S_{k-1}||_F^2 + 2 Re sum_{l<k} (u_l^H u_k)(v_l^H v_k)
  + ||u_k||^2 ||v_k||^2, and the iteration stops once
  ||u_k|| ||v_k|| <= eps ||S_k||_F;
* the next pivot row maximises |u_k| over rows not used yet;
* a residual row that is exactly zero is skipped (next unused row).

If the rank would reach m n / (m + n), where a low-rank pair stops saving
storage, the block is evaluated in full and truncated by its SVD instead.

Re-compression: U = Q_U R_U, V = Q_V R_V, R_U R_V^T = W diag(s) Y^H; keep
the smallest r' with (sum_{i >= r'} s_i^2)^(1/2) <= eps ||s||_2, giving
U' = Q_U W_r' diag(s_r'), V' = Q_V conj(Y_r') with Z_sub ~= U' V'^T.
"""

import numpy as np


def _truncation_rank(s, eps):
    tot = np.sqrt(np.sum(s * s))
    if tot == 0.0:
        return 0
    tail = np.sqrt(np.cumsum((s * s)[::-1])[::-1])   # tail[i] = ||s[i:]||
    for r in range(len(s) + 1):
        t = tail[r] if r < len(s) else 0.0
        if t <= eps * tot:
            return r
    return len(s)


def svd_truncate(block, eps):
    W, s, Yh = np.linalg.svd(block, full_matrices=False)
    r = _truncation_rank(s, eps)
    return W[:, :r] * s[:r], Yh[:r].T.copy()


def recompress(U, V, eps):
    if U.shape[1] == 0:
        return U, V
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(V)
    W, s, Yh = np.linalg.svd(Ru @ Rv.T)
    r = _truncation_rank(s, eps)
    return Qu @ (W[:, :r] * s[:r]), Qv @ Yh[:r].T


def aca(get_row, get_col, get_block, m, n, eps):
    """Return (U (m, r), V (n, r)) with block ~= U V^T."""
    limit = (m * n) / float(m + n)
    kmax = int(limit) + 1
    U = np.zeros((m, kmax), dtype=np.complex128)
    V = np.zeros((n, kmax), dtype=np.complex128)
    k = 0
    used = np.zeros(m, dtype=bool)
    i = 0
    norm2 = 0.0
    while True:
        if k + 1 >= limit:
            return svd_truncate(get_block(), eps)
        row = np.array(get_row(i), dtype=np.complex128) - V[:, :k] @ U[i, :k]
        used[i] = True
        j = int(np.argmax(np.abs(row)))
        if row[j] == 0.0:
            free = np.nonzero(~used)[0]
            if len(free) == 0:
                break
            i = int(free[0])
            continue
        v = row / row[j]
        u = np.array(get_col(j), dtype=np.complex128) - U[:, :k] @ V[j, :k]
        cross = np.sum((U[:, :k].conj().T @ u) * (V[:, :k].conj().T @ v))
        nu2 = np.vdot(u, u).real
        nv2 = np.vdot(v, v).real
        norm2 += 2.0 * cross.real + nu2 * nv2
        U[:, k] = u
        V[:, k] = v
        k += 1
        if np.sqrt(nu2 * nv2) <= eps * np.sqrt(norm2):
            break
        if np.all(used):
            break
        cand = np.abs(u)
        cand[used] = -1.0
        i = int(np.argmax(cand))
    return recompress(U[:, :k].copy(), V[:, :k].copy(), eps)
