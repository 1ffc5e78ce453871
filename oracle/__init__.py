"""Python driver for the FP64 oracle (``vrm_oracle.c``).

TEST INFRASTRUCTURE ONLY: this package may be imported by the test suite, the
smoke check and the benchmark's CPU-baseline leg, never by the product path.
It shares no code with the HIP library; it is a plain, serial-per-particle
restatement of the method of Kirchhart & Obi (see the C file's header for the
passages each piece follows and the readings taken where the paper is silent).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vrm_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libvrm_oracle.so")

KMAX = 48
NSEG = 8
STATUS_SMALL, STATUS_FULL, STATUS_INFEASIBLE, STATUS_NOT_DIFFUSED = 0, 1, 2, 3

# Shu-Osher SSP-RK3 weights and stage times (Sec. 3.3: convex combinations of Euler steps)
RK3_A = (0.0, 0.75, 1.0 / 3.0)
RK3_B = (1.0, 0.25, 2.0 / 3.0)
RK3_C = (0.0, 1.0, 0.5)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP contraction off so FP32 decisions are exact)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("nu", ctypes.c_double), ("r", ctypes.c_double),
                ("R", ctypes.c_double), ("R_full", ctypes.c_double), ("c_diff", ctypes.c_double),
                ("dt", ctypes.c_double), ("q", ctypes.c_int), ("solver", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def params(h, nu=0.01, q=2, r=0.5, R=2.0, R_full=None, c_diff=1.0, dt=0.0, solver=0) -> _Params:
    """solver 0: the canonical LP stencil; 1: non-negative least squares (Lawson-Hanson)."""
    if R_full is None:
        R_full = R if q == 2 else 3.0
    return _Params(h, nu, r, R, R_full, c_diff, dt, q, solver)


def params_of(wl, solver=0) -> _Params:
    return _Params(wl.h, wl.nu, wl.r, wl.R, wl.R_full, wl.c_diff, wl.dt, wl.q, solver)


def nnls(A: np.ndarray, b: np.ndarray):
    """min_{f >= 0} |A f - b|^2 (Lawson-Hanson) -> (f, additions) or raises on a rank-deficient subproblem."""
    A = np.ascontiguousarray(A, np.float64)
    m, k = A.shape
    f = np.zeros(k)
    adds = lib().orc_nnls(m, k, _p(A), _p(np.ascontiguousarray(b, np.float64)), _p(f))
    if adds < 0:
        raise RuntimeError("orc_nnls: rank-deficient subproblem")
    return f, adds


def rows(q: int) -> int:
    return 5 if q == 2 else 9


def moment_rhs(q: int) -> np.ndarray:
    b = np.zeros(rows(q))
    b[2] = b[4] = 2.0
    return b


# ------------------------------------------------------------------ pieces
def lp(A: np.ndarray, b: np.ndarray, c: np.ndarray):
    """min c.f s.t. A f = b, f >= 0 (dense two-phase simplex, Bland's rule). -> (status, f, pivots)."""
    A = np.ascontiguousarray(A, np.float64)
    m, k = A.shape
    f = np.zeros(k)
    basis = np.zeros(m, np.int32)
    piv = ctypes.c_int(0)
    st = lib().orc_lp(m, k, _p(A), _p(np.ascontiguousarray(b, np.float64)),
                      _p(np.ascontiguousarray(c, np.float64)), _p(f), _p(basis), ctypes.byref(piv))
    return st, f, piv.value


def diffused(gamma, ids, h, q, c_diff=1.0):
    """Sec. 3.5 reduced operator: mask of diffused particles, ||Gamma||_1 and the bound."""
    g = np.ascontiguousarray(gamma, np.float64)
    ids = np.ascontiguousarray(ids, np.int32)
    out = np.zeros(g.shape[0], np.uint8)
    n1, bd = ctypes.c_double(0), ctypes.c_double(0)
    lib().orc_diffused(g.shape[0], _p(g), _p(ids), ctypes.c_double(h), q, ctypes.c_double(c_diff),
                       _p(out), ctypes.byref(n1), ctypes.byref(bd))
    return out, n1.value, bd.value


@dataclass
class Stencils:
    kcol: np.ndarray
    cols: np.ndarray     # [n, KMAX] particle indices
    f: np.ndarray        # [n, KMAX] normalised fractions
    fii: np.ndarray
    status: np.ndarray
    small: np.ndarray    # [n, 8]
    kfull: np.ndarray
    pivots: int


def stencils(x, y, ids, mask, P: _Params) -> Stencils:
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    ids = np.ascontiguousarray(ids, np.int32)
    mask = np.ascontiguousarray(mask, np.uint8)
    n = x.shape[0]
    kcol = np.zeros(n, np.int32)
    cols = np.full((n, KMAX), -1, np.int32)
    f = np.zeros((n, KMAX))
    fii = np.zeros(n)
    status = np.zeros(n, np.uint8)
    small = np.zeros((n, NSEG), np.int32)
    kfull = np.zeros(n, np.int32)
    piv = ctypes.c_int64(0)
    err = lib().orc_stencils(n, _p(x), _p(y), _p(ids), _p(mask), ctypes.byref(P), _p(kcol), _p(cols),
                             _p(f), _p(fii), _p(status), _p(small), _p(kfull), ctypes.byref(piv))
    if err != 0:
        raise RuntimeError(f"orc_stencils failed ({err})")
    return Stencils(kcol, cols, f, fii, status, small, kfull, piv.value)


def apply(st: Stencils, gamma, P: _Params) -> np.ndarray:
    g = np.ascontiguousarray(gamma, np.float64)
    out = np.zeros_like(g)
    lib().orc_apply(g.shape[0], _p(st.kcol), _p(st.cols), _p(st.f), _p(st.fii), _p(st.status), _p(g),
                    ctypes.byref(P), _p(out))
    return out


def insert(x, y, gamma, ids, mask, P: _Params, capacity=None):
    """Sec. 4.2 insertion; returns (x, y, gamma, ids, n_candidates) with appended particles."""
    n = x.shape[0]
    cap = capacity or (n * 9 + 16)
    X = np.zeros(cap); X[:n] = x
    Y = np.zeros(cap); Y[:n] = y
    G = np.zeros(cap); G[:n] = gamma
    I = np.zeros(cap, np.int32); I[:n] = ids
    nc = ctypes.c_int32(0)
    nn = lib().orc_insert(n, cap, _p(X), _p(Y), _p(G), _p(I), _p(np.ascontiguousarray(mask, np.uint8)),
                          ctypes.byref(P), int(ids.max()) + 1 if n else 0, ctypes.byref(nc))
    if nn < 0:
        raise RuntimeError(f"orc_insert failed ({nn})")
    return X[:nn].copy(), Y[:nn].copy(), G[:nn].copy(), I[:nn].copy(), nc.value


@dataclass
class Removal:
    x: np.ndarray        # the cloud after removal (kept particles, in input order)
    y: np.ndarray
    gamma: np.ndarray
    ids: np.ndarray
    removed_ids: np.ndarray
    n_candidates: int
    kcol: np.ndarray     # per input particle: columns of its identity LP (removed ones)
    cols: np.ndarray     # [n, KMAX] input indices
    g: np.ndarray        # [n, KMAX] fractions


def remove(x, y, gamma, ids, P: _Params) -> Removal:
    """Sec. 6 (Outlook) particle removal: particles closer than r h to another
    are taken greedily in id order (none within R_full h of another taken one);
    each gives its circulation to its neighbours by the first-order identity
    LP (sum g = 1, sum g r = 0, g >= 0, min sum g (|r/h|^2 + 2^-16 rank^2)) and is
    dropped; one whose LP is infeasible stays."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    G = np.array(gamma, np.float64)
    ids = np.ascontiguousarray(ids, np.int32)
    n = x.shape[0]
    removed = np.zeros(n, np.uint8)
    kcol = np.zeros(n, np.int32)
    cols = np.full((n, KMAX), -1, np.int32)
    g = np.zeros((n, KMAX))
    nc = ctypes.c_int32(0)
    nr = lib().orc_remove(n, _p(x), _p(y), _p(G), _p(ids), ctypes.byref(P), _p(removed), _p(kcol), _p(cols),
                          _p(g), ctypes.byref(nc))
    if nr < 0:
        raise RuntimeError(f"orc_remove failed ({nr})")
    keep = removed == 0
    return Removal(x[keep].copy(), y[keep].copy(), G[keep].copy(), ids[keep].copy(), ids[~keep].copy(),
                   nc.value, kcol, cols, g)


def stencil_matrix_row(st: Stencils, i: int):
    """Column particle indices and fractions of particle i (incl. the self fraction)."""
    k = st.kcol[i]
    return st.cols[i, :k].copy(), st.f[i, :k].copy(), st.fii[i]


# --------------------------------------------------------------- full run
@dataclass
class StepInfo:
    n: int
    n_diffused: int
    n_inserted: int
    status_counts: list
    i0: float
    seconds: float = 0.0
    redistributed_gamma: float = 0.0   # sum of Gamma^n over the particles that redistributed (Euler steps)


@dataclass
class OracleState:
    x: np.ndarray
    y: np.ndarray
    gamma: np.ndarray
    ids: np.ndarray
    t: float
    history: list = field(default_factory=list)


def initial_state(wl) -> OracleState:
    return OracleState(wl.x.astype(np.float64), wl.y.astype(np.float64), wl.gamma.astype(np.float64),
                       np.arange(wl.n, dtype=np.int32), wl.t0)


def step(state: OracleState, wl, insertion: bool = True, record: bool = True, stages_cb=None,
         velocity=None, params=None) -> OracleState:
    """One SSP-RK3 step: diffused set and insertion at t^n, then three stages.
    velocity(x, y, gamma, t) -> (u, v) replaces the workload's prescribed field
    (for instance the particles' own Biot-Savart velocity, Sec. 3.4 eq. nsode);
    params (default params_of(wl)) selects the stencil solver."""
    P = params_of(wl) if params is None else params
    t_start = time.perf_counter()
    mask, _, _ = diffused(state.gamma, state.ids, wl.h, wl.q, wl.c_diff)
    n_before = state.x.shape[0]
    if insertion:
        x, y, g, ids, _ = insert(state.x, state.y, state.gamma, state.ids, mask, P)
        mask = np.concatenate([mask, np.zeros(x.shape[0] - n_before, np.uint8)])
    else:
        x, y, g, ids = state.x, state.y, state.gamma, state.ids
    x0, y0, g0 = x.copy(), y.copy(), g.copy()
    counts = [0, 0, 0]
    for s in range(3):
        ts = state.t + RK3_C[s] * wl.dt
        u, v = wl.velocity(x, y, ts) if velocity is None else velocity(x, y, g, ts)
        st = stencils(x, y, ids, mask, P)
        if stages_cb is not None:
            stages_cb(s, x, y, g, ids, mask, st)
        dg = apply(st, g, P)
        for c in range(3):
            counts[c] += int(np.count_nonzero(st.status == c))
        a, b = RK3_A[s], RK3_B[s]
        xn = a * x0 + b * (x + wl.dt * u)
        yn = a * y0 + b * (y + wl.dt * v)
        gn = a * g0 + b * (g + wl.dt * dg)
        x, y, g = xn, yn, gn
    out = OracleState(x, y, g, ids, state.t + wl.dt, state.history)
    if record:
        out.history.append(StepInfo(x.shape[0], int(mask.sum()), x.shape[0] - n_before, counts,
                                    float(g.sum()), time.perf_counter() - t_start))
    return out


def biot_savart(x, y, gamma, eps, tx=None, ty=None, chunk=256):
    """Velocity by the Biot-Savart law of the particles (Sec. 3.4, eq. nsode: dx_i/dt =
    sum_j K(r_ij) Gamma_j with r_ij = x_j - x_i) with the regularised kernel of Sec. 5,
    K_eps(d) = (-d_y, d_x) / (2 pi |d|^2) (1 - exp(-|d|^2 / eps^2)), d = x_i - x_j, and
    K_eps(0) = 0; at the particles, or at the points (tx, ty).  FP64, direct sum."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    g = np.asarray(gamma, np.float64)
    tx = x if tx is None else np.asarray(tx, np.float64)
    ty = y if ty is None else np.asarray(ty, np.float64)
    u = np.zeros(tx.shape[0])
    v = np.zeros(tx.shape[0])
    for a in range(0, tx.shape[0], chunk):
        dx = tx[a:a + chunk, None] - x[None, :]
        dy = ty[a:a + chunk, None] - y[None, :]
        r2 = dx * dx + dy * dy
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.where(r2 > 0.0, -np.expm1(-r2 / (eps * eps)) / (2.0 * np.pi * r2), 0.0)
        u[a:a + chunk] = (-dy * w) @ g
        v[a:a + chunk] = (dx * w) @ g
    return u, v


def euler_step(state: OracleState, wl, record: bool = True) -> OracleState:
    """One step of Euler's method for the heat equation (Sec. 3.3; the case without
    convection of Sec. 5): diffused set and insertion at t^n, then
    Gamma^{n+1} = Gamma^n + dt * nu sum_j f_ji Gamma_j^n on the new cloud; the
    particles do not move."""
    P = params_of(wl)
    t_start = time.perf_counter()
    mask, _, _ = diffused(state.gamma, state.ids, wl.h, wl.q, wl.c_diff)
    n_before = state.x.shape[0]
    x, y, g, ids, _ = insert(state.x, state.y, state.gamma, state.ids, mask, P)
    mask = np.concatenate([mask, np.zeros(x.shape[0] - n_before, np.uint8)])
    st = stencils(x, y, ids, mask, P)
    g_new = g + wl.dt * apply(st, g, P)
    out = OracleState(x, y, g_new, ids, state.t + wl.dt, state.history)
    if record:
        counts = [int(np.count_nonzero(st.status == c)) for c in range(3)]
        out.history.append(StepInfo(x.shape[0], int(mask.sum()), x.shape[0] - n_before, counts, float(g_new.sum()),
                                    time.perf_counter() - t_start, float(g[st.status < 2].sum())))
    return out


def run_euler(wl, steps=None) -> OracleState:
    st = initial_state(wl)
    for _ in range(wl.steps if steps is None else steps):
        st = euler_step(st, wl)
    return st


def run(wl, steps=None, insertion=True, solver=0) -> OracleState:
    """steps of SSP-RK3 from the workload's cloud; solver as in params()."""
    P = params_of(wl, solver=solver)
    st = initial_state(wl)
    for _ in range(wl.steps if steps is None else steps):
        st = step(st, wl, insertion=insertion, params=P)
    return st


def invariants(x, y, g):
    """I0, I1 and I2 of Sec. 3.4 (sums over particles, FP64)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    g = np.asarray(g, np.float64)
    return float(g.sum()), (float((g * x).sum()), float((g * y).sum())), float((g * (x * x + y * y)).sum())
