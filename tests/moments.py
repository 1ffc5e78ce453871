"""Moment residual of stencils recomputed on the host (test helper).

Sec. 2 eqs. (cond_two), (cond_alpha): a stencil f_ij of particle i must satisfy
sum_j fhat_ij rhat_ij^alpha = b_alpha for 1 <= |alpha| <= q, rhat = (x_j - x_i) / h,
b = 2 at alpha = (2, 0), (0, 2) and 0 otherwise.  The residual of a stencil is
max_alpha |sum_j fhat_ij rhat^alpha - b_alpha| / 2, in FP64 from the FP32
positions and fractions.  Written here from those definitions with numpy,
independently of the library's verification kernel, so that the kernel's report
can be checked against it.
"""
import numpy as np

ST_SMALL, ST_FULL, ST_WARM = 0, 1, 4


def stencil_columns(S, rows=None):
    """Column indices and fractions [m, K] of the stencils in S (numpy arrays
    small_idx [n, 8], small_f, status, full_k, full_idx [n, 48], full_f), for the
    given rows (default all) with a solved stencil; -1 columns are unused."""
    st = S["status"] if rows is None else S["status"][rows]
    rows = np.arange(st.size) if rows is None else np.asarray(rows)
    fk = S["full_k"][rows]
    small = (st == ST_SMALL) | ((st == ST_WARM) & (fk == 0))
    full = (st == ST_FULL) | ((st == ST_WARM) & (fk > 0))
    K = S["full_idx"].shape[1] if S.get("full_idx") is not None else 8
    cols = np.full((rows.size, K), -1, np.int64)
    f = np.zeros((rows.size, K))
    cols[small, :8] = S["small_idx"][rows[small]]
    f[small, :8] = S["small_f"][rows[small]]
    if S.get("full_idx") is not None:
        fr = rows[full]
        k = np.arange(K)[None, :] < fk[full][:, None]
        cols[full] = np.where(k, S["full_idx"][fr], -1)
        f[full] = np.where(k, S["full_f"][fr], 0.0)
    solved = small | full
    return rows[solved], cols[solved], f[solved]


def residuals(x, y, h, q, rows, cols, f):
    """Residual of each stencil (particle rows[a], columns cols[a], fractions f[a])."""
    x = np.asarray(x, np.float32).astype(np.float64)
    y = np.asarray(y, np.float32).astype(np.float64)
    f = np.asarray(f, np.float32).astype(np.float64)
    ok = cols >= 0
    c = np.where(ok, cols, 0)
    f = np.where(ok, f, 0.0)
    rx = (x[c] - x[rows][:, None]) / h
    ry = (y[c] - y[rows][:, None]) / h
    mono = [rx, ry, rx * rx, rx * ry, ry * ry]
    if q == 3:
        mono += [rx * rx * rx, rx * rx * ry, rx * ry * ry, ry * ry * ry]
    b = np.zeros(len(mono))
    b[2] = b[4] = 2.0
    res = np.zeros(rows.size)
    for a, v in enumerate(mono):
        res = np.maximum(res, np.abs((f * v).sum(axis=1) - b[a]) / 2.0)
    return res
