"""Autotuner of libvrm's launch shapes (the fields of vrm_tuning).

Times whole SSP-RK3 steps (vrm_step, graph replay) on the GPU for candidate
values of one field at a time, keeping the others at their current best
(coordinate descent, a fixed number of sweeps), and writes the fastest
configuration of each workload to tuning/<workload>.json, which bench.py
applies.  Each candidate runs from the same initial cloud: one untimed step,
then `steps` timed steps.  Launch shapes never change results.

    python -m paper_1508_06379_amd.autotune --workload lamb_oseen_h0.01_q2
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_DIR = os.path.join(HERE, "tuning")

# candidate values per field (0 = the library default); full_stored_cost_n:
# -1 never keep costs in LDS, 2^30 always
CANDIDATES = {
    "lp_small_blocks": [512, 1024, 2048, 4096, 8192],
    "lp_full_blocks": [256, 512, 768, 1024, 2048, 4096],
    "full_stored_cost_n": [-1, 200000, 1 << 30],
    "lp_small_lanes": [8, 16, 32, 64],
    "lp_small_coop": [1],
}


def tuning_path(workload: str) -> str:
    return os.path.join(TUNING_DIR, f"{workload}.json")


def load(workload: str):
    """The stored configuration of a workload, or None."""
    p = tuning_path(workload)
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        return json.load(fh)["tuning"]


def time_steps(wl, tuning: dict, steps: int, warm_mode: int = 0) -> float:
    """Mean ms per step of `steps` graph-replayed steps after one untimed step."""
    import torch
    import paper_1508_06379_amd as vrm
    P = vrm.params_of(wl)
    cap = int(wl.n * (4 if wl.n < 200000 else 2.2)) + 1024
    cloud = vrm.Cloud(wl.x, wl.y, wl.gamma, capacity=cap)
    ctx = vrm.Context(cap)
    ctx.vrm_set_tuning(tuning)
    if warm_mode:
        ctx.vrm_set_warm_start(warm_mode)
    vt = vrm.vortex_table(wl.vortices) if wl.vortices is not None else None
    t = wl.t0
    ctx.vrm_step(cloud, P, vt, t)
    t += wl.dt
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.vrm_step(cloud, P, vt, t)
        t += wl.dt
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    del ctx, cloud
    return ms


def relevant_fields(wl):
    """Fields that act on the workload's launches."""
    return ["lp_small_coop", "lp_small_lanes", "lp_small_blocks"] if wl.q == 2 else ["lp_full_blocks",
                                                                                     "full_stored_cost_n"]


def tune(name: str, wl, steps: int, sweeps: int = 2, warm_mode: int = 0, log=print) -> dict:
    import paper_1508_06379_amd as vrm
    best = {k: 0 for k in vrm.vrm_tuning.FIELDS}
    best_ms = time_steps(wl, best, steps, warm_mode)
    log(f"{name}: defaults {best_ms:.4f} ms/step")
    trials = [{"tuning": dict(best), "ms_per_step": best_ms}]
    for sweep in range(sweeps):
        changed = False
        for field in relevant_fields(wl):
            for v in CANDIDATES[field]:
                cand = dict(best, **{field: v})
                if cand == best:
                    continue
                ms = time_steps(wl, cand, steps, warm_mode)
                trials.append({"tuning": cand, "ms_per_step": ms})
                log(f"  sweep {sweep} {field}={v}: {ms:.4f} ms/step")
                if ms < best_ms * 0.99:   # a change must win by more than noise
                    best, best_ms, changed = cand, ms, True
        if not changed:
            break
    return {"tuning": best, "ms_per_step": best_ms, "steps_timed": steps, "warm_start": warm_mode,
            "trials": trials}


def main():
    sys.path.insert(0, os.path.dirname(HERE))
    import workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, choices=sorted(workloads.BENCH))
    ap.add_argument("--steps", type=int, default=0, help="timed steps per candidate (0: by workload size)")
    ap.add_argument("--sweeps", type=int, default=2)
    ap.add_argument("--out", default=None, help="output file (default tuning/<workload>.json)")
    args = ap.parse_args()
    wl = workloads.BENCH[args.workload]()
    steps = args.steps or (20 if wl.n < 200000 else (4 if wl.n < 5_000_000 else 1))
    res = tune(args.workload, wl, steps, args.sweeps, log=lambda m: print(m, flush=True))
    out = args.out or tuning_path(args.workload)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(f"best {res['tuning']} {res['ms_per_step']:.4f} ms/step -> {out}", flush=True)


if __name__ == "__main__":
    main()
