"""Throughput of the vorticity redistribution hot path on one MI355X.

A step is one SSP-RK3 step of the whole path: reduced-operator selection,
insertion and reordering (once per step), then for each of the three stages
the cell list, the small neighbourhoods, the moment LPs (small, then complete
neighbourhood fallback), the scatter of nu sum_j f_ji Gamma_j and the stage
combination.  The metric counts the stencils found and applied per second.

Prints ONE JSON line on stdout (everything else goes to stderr).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# MI355X published peaks and the VALU peak of non-packed FP32 (the design doc derives it)
PEAK_HBM_GBS = 8000.0
PEAK_FP32_NONPACKED_TFLOPS = 78.6

# algorithmic bytes per particle of the memory-bound kernel groups
BYTES_PER_PARTICLE = {
    "cells": 36.0,     # read x, y, id; write cell, rank, perm and x, y, id in slot order
    "nbhd": 42.0,      # own x, y, id, diffused; small neighbourhood (8 x 4 B) and a queue entry
    "combine": 40.0,   # read x0, y0, g0, x, y, g, u, v, acc; write x, y, g, acc (heat: no x/u traffic)
    "select": 20.0,    # four passes over |Gamma| and the mask
}

WORKLOADS = {
    "lamb_oseen_h0.01_q2": lambda: workloads.config_jittered(h=0.01, q=2, seed=2),
    "lamb_oseen_h0.01_q3": lambda: workloads.config_jittered(h=0.01, q=3, seed=2),
    "vortices64_h0.005": lambda: workloads.config_vortices(),
    "vortices256_h0.004_q3": lambda: workloads.config_scale(),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(wl, steps, warmup, theta=None):
    import torch
    import paper_1508_06379_amd as vrm

    torch.cuda.set_device(0)
    P = vrm.params_of(wl)
    cap = int(wl.n * (4 if wl.n < 200000 else 2.2)) + 1024
    cloud = vrm.Cloud(wl.x, wl.y, wl.gamma, capacity=cap)
    ctx = vrm.Context(cap)
    if theta is not None:
        ctx.vrm_mlp_load(theta)
        ctx.vrm_set_warm_start(True)
    vt = vrm.vortex_table(wl.vortices) if wl.vortices is not None else None

    t = wl.t0
    for _ in range(warmup):
        ctx.vrm_step(cloud, P, vt, t)
        t += wl.dt
    torch.cuda.synchronize()
    c0 = ctx.vrm_read_counters()
    n0 = cloud.n
    ctx.vrm_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.vrm_step(cloud, P, vt, t)
        t += wl.dt
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timers, overflow = ctx.vrm_read_timing()
    ctx.vrm_timing(False)
    c1 = ctx.vrm_read_counters()
    d = {k: c1[k] - c0[k] for k in ("redistributions", "pivots", "n_small", "n_full", "n_infeasible",
                                     "n_uncertified", "full_cols", "warm_hit", "warm_phase2", "warm_cold")}
    return dict(elapsed=elapsed, counters=d, timers=timers, timer_overflow=overflow, n_start=n0, n_end=cloud.n,
                final=c1)


def roofline(wl, res):
    """Roofline of the kernel group with the largest time in the timed region."""
    T = res["timers"]
    cand = {k: v for k, v in T.items() if k not in ("insert",) and v[1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    ms, launches = cand[dom]
    avg_s = ms / 1e3 / launches
    c = res["counters"]
    m = 5 if wl.q == 2 else 9
    if dom in ("lp_small", "lp_full"):
        # dense tableau simplex: one multiply-add per tableau entry and pivot,
        # tableau m x (k + 1); k = 8 (small) or the mean complete-neighbourhood size
        nlp = c["n_small"] if dom == "lp_small" else max(1, c["n_full"])
        k = 8.0 if dom == "lp_small" else c["full_cols"] / max(1, c["n_full"])
        flops = c["pivots"] * 2.0 * m * (k + 1.0)
        per_launch = flops / launches
        ach = per_launch / avg_s / 1e12
        return {"kernel": dom, "bound": "alu", "achieved": ach, "peak": PEAK_FP32_NONPACKED_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_NONPACKED_TFLOPS, "traffic": None,
                "avg_launch_ms": avg_s * 1e3, "launches": launches,
                "flop_model": f"pivots x 2 m (k+1), m={m}, k={k:.2f}, {c['pivots'] / max(1, nlp):.2f} pivots/LP"}
    npart = 0.5 * (res["n_start"] + res["n_end"])
    per_launch = BYTES_PER_PARTICLE[dom] * npart
    ach = per_launch / avg_s / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": None, "avg_launch_ms": avg_s * 1e3, "launches": launches}


def cpu_baseline(wl, budget_s=15.0, max_steps=100):
    """The FP64 oracle on the host cores, on the first steps of the same run."""
    import oracle
    oracle.build()
    st = oracle.initial_state(wl)
    red = 0
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps and time.perf_counter() - t0 < budget_s:
        st = oracle.step(st, wl)
        h = st.history[-1]
        red += h.status_counts[0] + h.status_counts[1]
        steps += 1
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": red / el, "unit": "redistributions/s", "cores": cores, "kind": "oracle",
            "sample": f"first {steps} SSP-RK3 steps of the same workload from its initial state "
                      f"({el:.1f} s; LPs and neighbourhoods OpenMP-parallel, insertion and apply serial)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lamb_oseen_h0.01_q2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the redistribution path has no multi-GPU mode "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    wl = WORKLOADS[args.workload]()
    log(f"workload {args.workload}: N={wl.n} h={wl.h} q={wl.q} dt={wl.dt}")
    res = run_gpu(wl, args.steps, args.warmup)
    c = res["counters"]
    value = c["redistributions"] / res["elapsed"]
    log(f"elapsed {res['elapsed']:.4f} s, counters {c}, timers {res['timers']}")
    rl = roofline(wl, res)
    line = {
        "metric": "particle redistributions/s (plain batched GPU solver), FP32, moments <= 1e-6",
        "value": value, "unit": "redistributions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["elapsed"] * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "h": wl.h, "q": wl.q, "n_start": res["n_start"],
                   "n_end": res["n_end"], "dt": wl.dt, "solver": "plain"},
        "roofline": rl,
        "timers_ms": {k: round(v[0], 4) for k, v in res["timers"].items()},
        "lp": {"small": c["n_small"], "full": c["n_full"], "infeasible": c["n_infeasible"],
               "uncertified": c["n_uncertified"], "pivots": c["pivots"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, budget_s=args.cpu_budget, max_steps=args.steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
