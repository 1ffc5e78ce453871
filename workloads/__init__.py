"""Seeded synthetic inputs for the vorticity-redistribution hot path.

This module is shared by the FP64 oracle, the tests and the benchmark.  It
holds only input generation: particle positions, the closed-form vorticity
fields they sample, and the closed-form velocity fields that the caller
supplies to each Runge-Kutta stage.  None of the redistribution method's own
arithmetic (neighbourhoods, moment conditions, linear programs, insertion,
time stepping) lives here.

Fields (Kirchhart & Obi, Sec. 5, Lamb-Oseen test case):
  * Lamb-Oseen vorticity  omega(t, x) = G / (4 pi nu t) exp(-|x|^2 / (4 nu t))
  * Lamb-Oseen velocity   u_theta(t, r) = G / (2 pi r) (1 - exp(-r^2 / (4 nu t)))
  * A Gaussian vortex with core sigma evolves as Lamb-Oseen with
    sigma^2 -> sigma^2 + 4 nu t; superpositions of such vortices give the
    multi-vortex fields (velocity prescribed, not induced).

All arrays are generated in float64 with numpy's PCG64 and cast once to
float32 (positions, circulations) or int32 (ids).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Workload", "lattice", "lamb_oseen_omega", "lamb_oseen_velocity",
    "vortex_set", "vortices_gamma", "vortices_velocity",
    "config_lattice_small", "config_jittered", "config_vortices",
    "config_scale", "config_close_pairs", "training_snapshot", "lone_particle", "PRESETS", "make", "BENCH",
    "c5_window",
]


@dataclasses.dataclass
class Workload:
    """One synthetic input state plus the run parameters that go with it."""
    name: str
    x: np.ndarray          # float32[N]
    y: np.ndarray          # float32[N]
    gamma: np.ndarray      # float32[N]
    h: float
    nu: float
    q: int                 # highest moment order matched (2 -> 5 rows, 3 -> 9 rows)
    dt: float
    steps: int
    t0: float = 0.0
    r: float = 0.5
    R: float = 2.0
    R_full: float = 2.0
    c_diff: float = 1.0
    vortices: Optional[dict] = None   # None -> zero velocity (heat equation)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def ids(self) -> np.ndarray:
        return np.arange(self.n, dtype=np.int32)

    def velocity(self, x, y, t):
        """Caller-supplied velocity at positions (x, y) and time t (float64)."""
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        if self.vortices is None:
            return np.zeros_like(x), np.zeros_like(y)
        return vortices_velocity(self.vortices, x, y, t, self.nu)


def lattice(lo: float, hi: float, h: float) -> tuple[np.ndarray, np.ndarray]:
    """Square lattice lo + i h, i = 0..round((hi - lo) / h), as float64 x, y (row-major in y)."""
    m = int(round((hi - lo) / h)) + 1
    g = lo + h * np.arange(m, dtype=np.float64)
    X, Y = np.meshgrid(g, g, indexing="xy")
    return X.ravel(), Y.ravel()


def lamb_oseen_omega(x, y, t, nu, gamma_total=1.0):
    """Lamb-Oseen vorticity at time t > 0 (Sec. 5)."""
    s = 4.0 * nu * t
    return gamma_total / (math.pi * s) * np.exp(-(x * x + y * y) / s)


def lamb_oseen_weak_error(x, y, g, t, nu, s=0.1):
    """Weak error of a particle field against the Lamb-Oseen vorticity at time t
    (Sec. 5.1): the largest |sum_i Gamma_i phi_c(x_i) - integral omega phi_c| over
    Gaussian test functions phi_c(x) = exp(-|x - c|^2 / s^2) centred on a 9 x 9 grid of
    c in [-0.4, 0.4]^2; the exact integral is s^2 / (s^2 + 4 nu t) exp(-|c|^2 / (s^2 + 4 nu t))
    (unit total circulation).  FP64."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    g = np.asarray(g, np.float64)
    a = 4.0 * nu * t
    err = 0.0
    for cx in np.linspace(-0.4, 0.4, 9):
        for cy in np.linspace(-0.4, 0.4, 9):
            num = (g * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / s ** 2)).sum()
            ex = s * s / (a + s * s) * np.exp(-(cx * cx + cy * cy) / (a + s * s))
            err = max(err, abs(num - ex))
    return err


def lamb_oseen_velocity(x, y, t, nu, gamma_total=1.0):
    """Lamb-Oseen velocity (counter-clockwise for positive circulation, Sec. 5)."""
    r2 = x * x + y * y
    s = 4.0 * nu * t
    with np.errstate(divide="ignore", invalid="ignore"):
        fac = np.where(r2 > 0, gamma_total / (2 * math.pi * r2) * (1 - np.exp(-r2 / s)), 0.0)
    return -fac * y, fac * x


def vortex_set(n_vortex: int, lo: float, hi: float, seed: int) -> dict:
    """Seeded Gaussian vortices: centres U[lo, hi]^2, cores U[0.2, 0.5], strengths N(0, 1)."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(lo, hi, n_vortex)
    cy = rng.uniform(lo, hi, n_vortex)
    sigma = rng.uniform(0.2, 0.5, n_vortex)
    g = rng.normal(0.0, 1.0, n_vortex)
    return {"cx": cx, "cy": cy, "sigma": sigma, "gamma": g}


_CHUNK = 1 << 20


def _chunked(fn, n, *arrays):
    """fn over consecutive chunks of the particle arrays on a few threads (numpy
    releases the interpreter lock in its loops); each particle's arithmetic, and
    so every result bit, is the same as in one pass."""
    if n <= _CHUNK:
        return fn(*arrays)
    from concurrent.futures import ThreadPoolExecutor
    import os
    bounds = [(a, min(a + _CHUNK, n)) for a in range(0, n, _CHUNK)]
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        parts = list(ex.map(lambda b: fn(*(arr[b[0]:b[1]] for arr in arrays)), bounds))
    if isinstance(parts[0], tuple):
        return tuple(np.concatenate([p[k] for p in parts]) for k in range(len(parts[0])))
    return np.concatenate(parts)


def vortices_gamma(v: dict, x, y, h: float, t: float = 0.0, nu: float = 0.0):
    """Particle circulations Gamma_i = omega(t, x_i) h^2 for a sum of Gaussian vortices."""
    def part(x, y):
        out = np.zeros_like(x, dtype=np.float64)
        for cx, cy, s, g in zip(v["cx"], v["cy"], v["sigma"], v["gamma"]):
            s2 = s * s + 4.0 * nu * t
            out += g / (math.pi * s2) * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / s2)
        return out * h * h
    return _chunked(part, np.asarray(x).shape[0], np.asarray(x), np.asarray(y))


def vortices_velocity(v: dict, x, y, t: float, nu: float):
    """Superposed Lamb-Oseen velocities of the spreading Gaussian vortices (prescribed field)."""
    def part(x, y):
        u = np.zeros_like(x, dtype=np.float64)
        w = np.zeros_like(y, dtype=np.float64)
        for cx, cy, s, g in zip(v["cx"], v["cy"], v["sigma"], v["gamma"]):
            dx = x - cx
            dy = y - cy
            r2 = dx * dx + dy * dy
            s2 = s * s + 4.0 * nu * t
            with np.errstate(divide="ignore", invalid="ignore"):
                fac = np.where(r2 > 0, g / (2 * math.pi * r2) * (1 - np.exp(-r2 / s2)), 0.0)
            u -= fac * dy
            w += fac * dx
        return u, w
    return _chunked(part, np.asarray(x).shape[0], np.asarray(x, np.float64), np.asarray(y, np.float64))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def config_lattice_small() -> Workload:
    """Lamb-Oseen at t0 = 1 sampled on the lattice -1 + i h, h = 0.05 (41^2 = 1681 particles)."""
    h, nu, t0 = 0.05, 0.01, 1.0
    x, y = lattice(-1.0, 1.0, h)
    g = lamb_oseen_omega(x, y, t0, nu) * h * h
    return Workload("lamb_oseen_lattice_h0.05", _f32(x), _f32(y), _f32(g), h=h, nu=nu, q=2,
                    dt=0.1 * h * h / nu, steps=10, t0=t0)


def config_jittered(h: float = 0.01, q: int = 2, seed: int = 2, steps: Optional[int] = None,
                    jitter: float = 0.25) -> Workload:
    """Lamb-Oseen at t0 = 1 on a lattice over [-1, 1]^2 jittered by U(+-jitter h) per coordinate."""
    nu, t0 = 0.01, 1.0
    x, y = lattice(-1.0, 1.0, h)
    rng = np.random.default_rng(seed)
    x = x + rng.uniform(-jitter * h, jitter * h, x.shape)
    y = y + rng.uniform(-jitter * h, jitter * h, y.shape)
    x32, y32 = _f32(x), _f32(y)
    g = lamb_oseen_omega(x32.astype(np.float64), y32.astype(np.float64), t0, nu) * h * h
    return Workload(f"lamb_oseen_jittered_h{h}_q{q}", x32, y32, _f32(g), h=h, nu=nu, q=q,
                    dt=0.1 * h * h / nu, steps=100 if steps is None else steps, t0=t0,
                    R_full=2.0 if q == 2 else 3.0)


def _vortex_cloud(name, lo, hi, h, n_vortex, seed_v, seed_jit, seed_del, p_delete, q):
    nu = 0.01
    x, y = lattice(lo, hi, h)
    rng = np.random.default_rng(seed_jit)
    x = x + rng.uniform(-0.4 * h, 0.4 * h, x.shape)
    y = y + rng.uniform(-0.4 * h, 0.4 * h, y.shape)
    if p_delete > 0:
        keep = np.random.default_rng(seed_del).random(x.shape) >= p_delete
        x, y = x[keep], y[keep]
    v = vortex_set(n_vortex, lo, hi, seed_v)
    x32, y32 = _f32(x), _f32(y)
    g = vortices_gamma(v, x32.astype(np.float64), y32.astype(np.float64), h)
    return Workload(name, x32, y32, _f32(g), h=h, nu=nu, q=q, dt=0.1 * h * h / nu, steps=10,
                    t0=0.0, R_full=2.0 if q == 2 else 3.0, vortices=v)


def config_vortices(h: float = 0.005, lo: float = -4.0, hi: float = 4.0) -> Workload:
    """64 Gaussian vortices, lattice jitter +-0.4h, 20% deletion, prescribed velocity, q = 2."""
    return _vortex_cloud(f"vortices64_h{h}", lo, hi, h, 64, 3, 31, 32, 0.2, 2)


def config_scale(h: float = 0.004, lo: float = -8.0, hi: float = 8.0, q: int = 3) -> Workload:
    """256 Gaussian vortices on [-8, 8]^2, h = 0.004 (16.0 M particles), jitter +-0.4h, no deletion."""
    w = _vortex_cloud(f"vortices256_h{h}_q{q}", lo, hi, h, 256, 5, 51, 0, 0.0, q)
    w.steps = 50
    return w


def config_close_pairs(h: float = 0.01, q: int = 2, frac: float = 0.05, seed: int = 4, lo: float = -1.0,
                       hi: float = 1.0) -> Workload:
    """Particle-removal input: the jittered Lamb-Oseen cloud (U(+-0.25h) per
    coordinate) over [lo, hi]^2 plus, at a seeded fraction `frac` of the sites,
    one more particle at distance U(0.05h, 0.45h) in a uniform direction (closer
    than r h = 0.5h to its site).  The extra particles carry the field's
    circulation density too and take the ids after the sites."""
    nu, t0 = 0.01, 1.0
    x, y = lattice(lo, hi, h)
    rng = np.random.default_rng(seed)
    x = x + rng.uniform(-0.25 * h, 0.25 * h, x.shape)
    y = y + rng.uniform(-0.25 * h, 0.25 * h, y.shape)
    pick = rng.random(x.shape) < frac
    d = rng.uniform(0.05 * h, 0.45 * h, int(pick.sum()))
    a = rng.uniform(0.0, 2.0 * np.pi, d.shape)
    x = np.concatenate([x, x[pick] + d * np.cos(a)])
    y = np.concatenate([y, y[pick] + d * np.sin(a)])
    x32, y32 = _f32(x), _f32(y)
    g = lamb_oseen_omega(x32.astype(np.float64), y32.astype(np.float64), t0, nu) * h * h
    return Workload(f"close_pairs_h{h}_q{q}", x32, y32, _f32(g), h=h, nu=nu, q=q, dt=0.1 * h * h / nu,
                    steps=0, t0=t0, R_full=2.0 if q == 2 else 3.0)


def training_snapshot(seed: int, h: float = 0.01, q: int = 2, kind: str = "lamb_oseen") -> Workload:
    """Training geometry with its own seed: the jittered Lamb-Oseen generator
    (kind "lamb_oseen"), or the vortex-cloud generator with lattice jitter
    +-0.4h and 20% deletion ("vortices") or none ("vortices_dense") over
    [-4, 4]^2.  Only offsets / h enter the network, so h sets the cloud size."""
    if kind == "lamb_oseen":
        return config_jittered(h=h, q=q, seed=seed, steps=0)
    p_delete = 0.2 if kind == "vortices" else 0.0
    return _vortex_cloud(f"train_{kind}_{seed}", -4.0, 4.0, h, 64, seed, seed + 7919, seed + 104729, p_delete, q)


def lone_particle(h: float = 0.05, gamma: float = 1.0) -> Workload:
    """A single circulation-carrying particle (the Dirac start of Sec. 5)."""
    z = np.zeros(1, np.float32)
    return Workload("dirac", z.copy(), z.copy(), np.array([gamma], np.float32), h=h, nu=0.02,
                    q=2, dt=0.1 * h * h / 0.02, steps=1)


def dirac_lamb_oseen(h: float) -> Workload:
    """The paper's Lamb-Oseen test with the heat equation (Sec. 5): a single particle
    of circulation 2 pi at the origin, nu = 1/50, C_diff = 1, q = 2, Euler steps of
    dt = (r h)^2 / (32 nu) with r = 1/2 up to t = 1 (2.56 / h^2 steps)."""
    nu = 1.0 / 50.0
    dt = (0.5 * h) ** 2 / (32.0 * nu)
    z = np.zeros(1, np.float32)
    return Workload(f"dirac_h{h}", z.copy(), z.copy(), np.array([2.0 * np.pi], np.float32), h=h, nu=nu, q=2,
                    dt=dt, steps=int(round(1.0 / dt)), t0=0.0)


# the benchmark's workloads by name (bench.py, the autotuner, the full-size tests)
BENCH = {
    "lamb_oseen_h0.01_q2": lambda: config_jittered(h=0.01, q=2, seed=2),
    "lamb_oseen_h0.01_q3": lambda: config_jittered(h=0.01, q=3, seed=2),
    "vortices64_h0.005": lambda: config_vortices(),
    "vortices256_h0.004_q3": lambda: config_scale(),
}


def c5_window(wl: Workload, half: float) -> Workload:
    """The particles of a vortex-cloud workload inside [-half, half]^2, with their
    circulations and the same prescribed velocity field (a bounded sample of the
    workload for the host-side reference timing)."""
    sel = (np.abs(wl.x) <= half) & (np.abs(wl.y) <= half)
    return dataclasses.replace(wl, name=f"{wl.name}_window{half}", x=wl.x[sel].copy(), y=wl.y[sel].copy(),
                               gamma=wl.gamma[sel].copy())


PRESETS = {
    "lattice": config_lattice_small,
    "jittered_q2": lambda: config_jittered(q=2),
    "jittered_q3": lambda: config_jittered(q=3),
    "vortices": config_vortices,
    "scale": config_scale,
}


def make(name: str) -> Workload:
    return PRESETS[name]()
