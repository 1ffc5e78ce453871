"""Python binding of libvrm, the MI355X (gfx950) vorticity redistribution library.

Argument marshalling only: every step of the method runs in the HIP kernels of
``libvrm.so`` (declared in ``include/vrm.h``).  PyTorch provides device memory
and the stream.  There is no CPU fallback: importing works without a GPU, but
every call needs the built library and a GPU, and raises otherwise.

Kirchhart & Obi, "A Splitting-free Vorticity Redistribution Method": the
library computes non-negative redistribution fractions under the moment
conditions (Sec. 2), inserts particles where a neighbourhood has an empty
segment (Sec. 4.2), and applies dGamma_i/dt = nu sum_j f_ji Gamma_j inside SSP
Runge-Kutta stages (Sec. 3.3-3.4).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvrm.so")

NSEG = 8
KMAX = 48
ST_SMALL, ST_FULL, ST_INFEASIBLE, ST_SKIPPED, ST_WARM = 0, 1, 2, 3, 4
E_ARG, E_CAPACITY, E_HIP, E_STATE, E_NONFINITE = -1, -2, -3, -4, -5


class VrmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class vrm_params(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("nu", ctypes.c_double), ("r", ctypes.c_double), ("R", ctypes.c_double),
                ("R_full", ctypes.c_double), ("c_diff", ctypes.c_double), ("dt", ctypes.c_double),
                ("q", ctypes.c_int32), ("deterministic", ctypes.c_int32)]


class vrm_tuning(ctypes.Structure):
    _fields_ = [("lp_small_blocks", ctypes.c_int32), ("lp_full_blocks", ctypes.c_int32),
                ("full_stored_cost_n", ctypes.c_int32), ("infer_blocks", ctypes.c_int32),
                ("lp_small_lanes", ctypes.c_int32), ("lp_small_coop", ctypes.c_int32), ("cert_rounds", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]
    FIELDS = ("lp_small_blocks", "lp_full_blocks", "full_stored_cost_n", "infer_blocks", "lp_small_lanes",
              "lp_small_coop", "cert_rounds")


class vrm_cloud(ctypes.Structure):
    _fields_ = [("x_dev", ctypes.c_void_p), ("y_dev", ctypes.c_void_p), ("gamma_dev", ctypes.c_void_p),
                ("id_dev", ctypes.c_void_p), ("n_dev", ctypes.c_void_p), ("capacity", ctypes.c_int32)]


class vrm_stencils(ctypes.Structure):
    _fields_ = [("small_idx_dev", ctypes.c_void_p), ("small_f_dev", ctypes.c_void_p), ("fii_dev", ctypes.c_void_p),
                ("status_dev", ctypes.c_void_p), ("full_k_dev", ctypes.c_void_p),
                ("full_idx_dev", ctypes.c_void_p), ("full_f_dev", ctypes.c_void_p)]


class vrm_counters(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_diffused", ctypes.c_int32), ("n_candidates", ctypes.c_int32),
                ("n_inserted", ctypes.c_int32), ("n_small", ctypes.c_int64), ("n_full", ctypes.c_int64),
                ("n_infeasible", ctypes.c_int64), ("n_uncertified", ctypes.c_int64),
                ("n_truncated", ctypes.c_int64), ("n_grid_clamped", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("pivots", ctypes.c_int64), ("redistributions", ctypes.c_int64),
                ("capacity_needed", ctypes.c_int32), ("mis_rounds", ctypes.c_int32), ("full_cols", ctypes.c_int64),
                ("warm_hit", ctypes.c_int64), ("warm_phase2", ctypes.c_int64), ("warm_cold", ctypes.c_int64),
                ("graph_replays", ctypes.c_int64), ("cert_rounds", ctypes.c_int64), ("cert_exact", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["vrm_create", "vrm_destroy", "vrm_select_diffused", "vrm_set_diffused", "vrm_build_neighbourhoods",
           "vrm_insert_particles", "vrm_remove_particles", "vrm_solve_fractions", "vrm_rk_stage", "vrm_step", "vrm_set_graph", "vrm_set_tuning",
           "vrm_get_tuning", "vrm_verify",
           "vrm_read_counters",
           "vrm_vortex_velocity", "vrm_biot_savart", "vrm_set_lp_objective", "vrm_timing", "vrm_timing_groups", "vrm_read_timing", "vrm_mlp_load", "vrm_mlp_read",
           "vrm_set_warm_start", "vrm_collect_training", "vrm_mlp_train_step", "vrm_mlp_infer", "vrm_gemm_bf16",
           "vrm_select_diffused_static", "vrm_warm_predictions", "vrm_last_error", "vrm_status_string"]
MLP_IN, MLP_OUT, MLP_PARAMS, MLP_SLOTS = 128, 64, 41280, 32
TIMERS = ["select", "cells", "nbhd", "lp_small", "lp_full", "insert", "combine", "mlp", "full_cols"]

_lib = None


def lib():
    """Load libvrm.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libvrm.so not built ({LIB_PATH}); run paper_1508_06379_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.vrm_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_int32]
        L.vrm_destroy.argtypes = [vp]
        L.vrm_select_diffused.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.POINTER(vrm_params), vp]
        L.vrm_set_diffused.argtypes = [vp, ctypes.POINTER(vrm_cloud), vp]
        L.vrm_build_neighbourhoods.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.POINTER(vrm_params), vp, vp]
        L.vrm_insert_particles.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.POINTER(vrm_params)]
        L.vrm_remove_particles.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.POINTER(vrm_params),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.vrm_solve_fractions.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.POINTER(vrm_params),
                                          ctypes.POINTER(vrm_stencils)]
        L.vrm_rk_stage.argtypes = [vp, ctypes.POINTER(vrm_cloud), vp, vp, ctypes.POINTER(vrm_params), ctypes.c_int]
        L.vrm_step.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.POINTER(vrm_params), vp, ctypes.c_int32,
                               ctypes.c_double]
        L.vrm_set_graph.argtypes = [vp, ctypes.c_int]
        L.vrm_set_tuning.argtypes = [vp, ctypes.POINTER(vrm_tuning)]
        L.vrm_get_tuning.argtypes = [vp, ctypes.POINTER(vrm_tuning)]
        L.vrm_verify.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.POINTER(vrm_params),
                                 ctypes.POINTER(vrm_stencils), vp]
        L.vrm_read_counters.argtypes = [vp, ctypes.POINTER(vrm_counters)]
        L.vrm_biot_savart.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.c_double, vp, vp]
        L.vrm_set_lp_objective.argtypes = [vp, ctypes.c_int]
        L.vrm_vortex_velocity.argtypes = [vp, ctypes.POINTER(vrm_cloud), vp, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_double, vp, vp]
        L.vrm_mlp_load.argtypes = [vp, vp]
        L.vrm_mlp_read.argtypes = [vp, vp]
        L.vrm_set_warm_start.argtypes = [vp, ctypes.c_int]
        L.vrm_collect_training.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.POINTER(vrm_params), vp, vp,
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.vrm_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         vp, vp]
        L.vrm_mlp_infer.argtypes = [vp, vp, ctypes.c_int32, vp]
        L.vrm_warm_predictions.argtypes = [vp, ctypes.POINTER(vrm_cloud), ctypes.POINTER(vrm_params), vp, vp,
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.vrm_gemm_bf16.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                    ctypes.c_int]
        L.vrm_timing.argtypes = [vp, ctypes.c_int]
        L.vrm_timing_groups.argtypes = [vp, ctypes.c_uint32]
        L.vrm_read_timing.argtypes = [vp, vp, vp]
        L.vrm_select_diffused_static.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                                 vp, vp, vp]
        L.vrm_last_error.restype = ctypes.c_char_p
        L.vrm_status_string.restype = ctypes.c_char_p
        L.vrm_status_string.argtypes = [ctypes.c_int]
        for name in EXPORTS:
            if name not in ("vrm_last_error", "vrm_status_string"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise VrmError(code, lib().vrm_last_error().decode())
    return code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def make_params(h, nu=0.01, q=2, dt=0.0, r=0.5, R=2.0, R_full=None, c_diff=1.0, deterministic=0) -> vrm_params:
    if R_full is None:
        R_full = R if q == 2 else 3.0
    return vrm_params(h, nu, r, R, R_full, c_diff, dt, q, int(deterministic))


def params_of(wl, deterministic=0) -> vrm_params:
    return vrm_params(wl.h, wl.nu, wl.r, wl.R, wl.R_full, wl.c_diff, wl.dt, wl.q, int(deterministic))


class Cloud:
    """Device particle cloud (torch tensors) with spare capacity for insertion."""

    def __init__(self, x, y, gamma, ids=None, capacity=None, device="cuda"):
        import torch
        n = len(x)
        cap = int(capacity or max(16, 2 * n))
        self.capacity = cap
        self.x = torch.zeros(cap, dtype=torch.float32, device=device)
        self.y = torch.zeros(cap, dtype=torch.float32, device=device)
        self.gamma = torch.zeros(cap, dtype=torch.float32, device=device)
        self.id = torch.zeros(cap, dtype=torch.int32, device=device)
        self.n_dev = torch.tensor([n], dtype=torch.int32, device=device)
        if n:
            self.x[:n] = torch.as_tensor(np.asarray(x, np.float32), device=device)
            self.y[:n] = torch.as_tensor(np.asarray(y, np.float32), device=device)
            self.gamma[:n] = torch.as_tensor(np.asarray(gamma, np.float32), device=device)
            ids = np.arange(n, dtype=np.int32) if ids is None else np.asarray(ids, np.int32)
            self.id[:n] = torch.as_tensor(ids, device=device)
        self.c = vrm_cloud(self.x.data_ptr(), self.y.data_ptr(), self.gamma.data_ptr(), self.id.data_ptr(),
                           self.n_dev.data_ptr(), cap)

    @property
    def n(self) -> int:
        return int(self.n_dev.item())

    def numpy(self):
        """(x, y, gamma, id) of the current particles, in array order."""
        n = self.n
        return (self.x[:n].cpu().numpy(), self.y[:n].cpu().numpy(), self.gamma[:n].cpu().numpy(),
                self.id[:n].cpu().numpy())


@dataclass
class Stencils:
    small_idx: object
    small_f: object
    fii: object
    status: object
    full_k: object
    full_idx: object
    full_f: object

    @staticmethod
    def alloc(capacity, full=True, device="cuda"):
        import torch
        z = lambda *s, dt=torch.float32: torch.zeros(*s, dtype=dt, device=device)
        return Stencils(z(capacity, NSEG, dt=torch.int32), z(capacity, NSEG), z(capacity),
                        z(capacity, dt=torch.uint8), z(capacity, dt=torch.int32),
                        z(capacity, KMAX, dt=torch.int32) if full else None, z(capacity, KMAX) if full else None)

    def c(self):
        return vrm_stencils(*[t.data_ptr() if t is not None else None for t in
                              (self.small_idx, self.small_f, self.fii, self.status, self.full_k, self.full_idx,
                               self.full_f)])


class Context:
    """A libvrm context on the current torch device and stream."""

    def __init__(self, capacity, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libvrm needs a GPU; none is visible")
        dev = torch.cuda.current_device() if device is None else device
        s = torch.cuda.current_stream(dev) if stream is None else stream
        self.stream = s
        self.handle = ctypes.c_void_p()
        _check(lib().vrm_create(ctypes.byref(self.handle), dev, ctypes.c_void_p(s.cuda_stream), int(capacity)))
        self.capacity = capacity

    def close(self):
        if self.handle:
            lib().vrm_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- entry points, same names as the C ABI
    def vrm_select_diffused(self, cloud: Cloud, p: vrm_params, mask=None):
        _check(lib().vrm_select_diffused(self.handle, ctypes.byref(cloud.c), ctypes.byref(p), _ptr(mask)))

    def vrm_set_diffused(self, cloud: Cloud, mask):
        _check(lib().vrm_set_diffused(self.handle, ctypes.byref(cloud.c), _ptr(mask)))

    def vrm_build_neighbourhoods(self, cloud: Cloud, p: vrm_params, small_idx=None, kfull=None):
        _check(lib().vrm_build_neighbourhoods(self.handle, ctypes.byref(cloud.c), ctypes.byref(p), _ptr(small_idx),
                                              _ptr(kfull)))

    def vrm_insert_particles(self, cloud: Cloud, p: vrm_params):
        _check(lib().vrm_insert_particles(self.handle, ctypes.byref(cloud.c), ctypes.byref(p)))

    def vrm_remove_particles(self, cloud: Cloud, p: vrm_params):
        """Particle removal (Sec. 6, outlook); returns (removed, candidates)."""
        nr, nc = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().vrm_remove_particles(self.handle, ctypes.byref(cloud.c), ctypes.byref(p), ctypes.byref(nr),
                                          ctypes.byref(nc)))
        return nr.value, nc.value

    def vrm_solve_fractions(self, cloud: Cloud, p: vrm_params, out: Stencils):
        st = out.c()
        _check(lib().vrm_solve_fractions(self.handle, ctypes.byref(cloud.c), ctypes.byref(p), ctypes.byref(st)))

    def vrm_rk_stage(self, cloud: Cloud, p: vrm_params, stage: int, u=None, v=None):
        _check(lib().vrm_rk_stage(self.handle, ctypes.byref(cloud.c), _ptr(u), _ptr(v), ctypes.byref(p), stage))

    def vrm_step(self, cloud: Cloud, p: vrm_params, vort=None, t=0.0):
        _check(lib().vrm_step(self.handle, ctypes.byref(cloud.c), ctypes.byref(p), _ptr(vort),
                              int(vort.shape[0]) if vort is not None else 0, float(t)))

    def vrm_set_tuning(self, tuning=None):
        """Launch shapes from a dict of vrm_tuning fields (missing or 0: default); None: defaults."""
        if tuning is None:
            _check(lib().vrm_set_tuning(self.handle, None))
            return
        t = vrm_tuning()
        for k, v in tuning.items():
            if k not in vrm_tuning.FIELDS:
                raise KeyError(k)
            setattr(t, k, int(v))
        _check(lib().vrm_set_tuning(self.handle, ctypes.byref(t)))

    def vrm_get_tuning(self) -> dict:
        t = vrm_tuning()
        _check(lib().vrm_get_tuning(self.handle, ctypes.byref(t)))
        return {k: getattr(t, k) for k in vrm_tuning.FIELDS}

    def vrm_set_graph(self, enable: bool):
        _check(lib().vrm_set_graph(self.handle, 1 if enable else 0))

    def vrm_verify(self, cloud: Cloud, p: vrm_params, st: Stencils, report):
        sc = st.c() if st is not None else None
        _check(lib().vrm_verify(self.handle, ctypes.byref(cloud.c), ctypes.byref(p),
                                ctypes.byref(sc) if sc is not None else None, _ptr(report)))

    def vrm_read_counters(self) -> dict:
        c = vrm_counters()
        _check(lib().vrm_read_counters(self.handle, ctypes.byref(c)))
        return c.as_dict()

    def vrm_set_lp_objective(self, mode: int):
        """0: the canonical stencil (default); 1: the first feasible vertex (phase I only)."""
        _check(lib().vrm_set_lp_objective(self.handle, int(mode)))

    def vrm_biot_savart(self, cloud: Cloud, eps, u, v):
        _check(lib().vrm_biot_savart(self.handle, ctypes.byref(cloud.c), ctypes.c_double(eps), _ptr(u), _ptr(v)))

    def vrm_vortex_velocity(self, cloud: Cloud, vort, nu, t, u, v):
        _check(lib().vrm_vortex_velocity(self.handle, ctypes.byref(cloud.c), _ptr(vort), int(vort.shape[0]),
                                         float(nu), float(t), _ptr(u), _ptr(v)))

    def vrm_timing(self, enable: bool):
        _check(lib().vrm_timing(self.handle, 1 if enable else 0))

    def vrm_timing_groups(self, groups):
        """Time only the named groups (an iterable of TIMERS names; empty: off)."""
        mask = 0
        for g in groups:
            mask |= 1 << TIMERS.index(g)
        _check(lib().vrm_timing_groups(self.handle, mask))

    def vrm_read_timing(self):
        """{group: (total ms, launches)} of the interval since the last read."""
        ms = (ctypes.c_double * len(TIMERS))()
        ln = (ctypes.c_int64 * len(TIMERS))()
        rc = lib().vrm_read_timing(self.handle, ms, ln)
        if rc < 0:
            _check(rc)
        return {k: (ms[i], ln[i]) for i, k in enumerate(TIMERS)}, rc == 1

    # --- learned warm start
    def vrm_mlp_load(self, params):
        _check(lib().vrm_mlp_load(self.handle, _ptr(params)))

    def vrm_mlp_read(self, params):
        _check(lib().vrm_mlp_read(self.handle, _ptr(params)))

    def vrm_set_warm_start(self, mode):
        """0/False off, 1/True from the network, 2 from each particle's previous basis."""
        _check(lib().vrm_set_warm_start(self.handle, int(mode)))

    def vrm_collect_training(self, cloud: Cloud, p: vrm_params, x, y) -> int:
        rows = ctypes.c_int32(0)
        _check(lib().vrm_collect_training(self.handle, ctypes.byref(cloud.c), ctypes.byref(p), _ptr(x), _ptr(y),
                                          int(x.shape[0]), ctypes.byref(rows)))
        return rows.value

    def vrm_mlp_train_step(self, x, y, rows, lr, weight_decay=0.0, frac_weight=1.0, loss=None, grad=None):
        _check(lib().vrm_mlp_train_step(self.handle, _ptr(x), _ptr(y), int(rows), float(lr), float(weight_decay),
                                        float(frac_weight), _ptr(loss), _ptr(grad)))

    def vrm_mlp_infer(self, x, rows, y):
        _check(lib().vrm_mlp_infer(self.handle, _ptr(x), int(rows), _ptr(y)))

    def vrm_warm_predictions(self, cloud: Cloud, p: vrm_params, out, particle) -> int:
        rows = ctypes.c_int32(0)
        _check(lib().vrm_warm_predictions(self.handle, ctypes.byref(cloud.c), ctypes.byref(p), _ptr(out),
                                          _ptr(particle), int(out.shape[0]), ctypes.byref(rows)))
        return rows.value

    def vrm_gemm_bf16(self, a, b, c, M, N, K, trans_a=False, trans_b=False):
        _check(lib().vrm_gemm_bf16(self.handle, _ptr(a), _ptr(b), _ptr(c), M, N, K, int(trans_a), int(trans_b)))

    # --- convenience
    def step(self, cloud: Cloud, p: vrm_params, velocity=None, t=0.0, insertion=True):
        """One SSP-RK3 step: insertion (diffused set, new particles, reorder), then three stages.
        velocity(cloud, t_stage) -> (u, v) device tensors or None for zero velocity."""
        if insertion:
            self.vrm_insert_particles(cloud, p)
        for s, c in enumerate((0.0, 1.0, 0.5)):
            uv = velocity(cloud, t + c * p.dt) if velocity is not None else None
            u, v = uv if uv is not None else (None, None)
            self.vrm_rk_stage(cloud, p, s, u, v)


def vrm_select_diffused_static(gamma, n: int, h: float, q: int, c_diff: float, mask, nonfinite=None, stream=None):
    """Sec. 3.5 selection without a context (allocates nothing): mask[:n] = 1 for the
    diffused particles of gamma[:n]; on the current torch device and stream."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    _check(lib().vrm_select_diffused_static(_ptr(gamma), int(n), float(h), int(q), float(c_diff), _ptr(mask),
                                            _ptr(nonfinite), ctypes.c_void_p(s.cuda_stream)))


def vortex_table(v: dict, device="cuda"):
    """Device table [n][4] (cx, cy, sigma, Gamma) for vrm_vortex_velocity."""
    import torch
    tab = np.stack([v["cx"], v["cy"], v["sigma"], v["gamma"]], 1).astype(np.float32)
    return torch.as_tensor(tab, device=device).contiguous()
