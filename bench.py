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

# MI355X published HBM peak; FP32 VALU peak without packed math: 256 CUs x 4 SIMDs
# x 16 lanes x 2 FLOP (FMA) x 2.4 GHz (the library emits no packed FP32)
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


def run_gpu(wl, steps, warmup, theta=None, warm_mode=0, tuning=None, lp_objective=0):
    import torch
    import paper_1508_06379_amd as vrm

    torch.cuda.set_device(0)
    P = vrm.params_of(wl)
    cap = int(wl.n * (4 if wl.n < 200000 else 2.2)) + 1024
    cloud = vrm.Cloud(wl.x, wl.y, wl.gamma, capacity=cap)
    ctx = vrm.Context(cap)
    if tuning:
        ctx.vrm_set_tuning(tuning)
    ctx.vrm_set_lp_objective(lp_objective)
    if theta is not None:
        ctx.vrm_mlp_load(theta)
        ctx.vrm_set_warm_start(1)
    elif warm_mode:
        ctx.vrm_set_warm_start(warm_mode)
    vt = vrm.vortex_table(wl.vortices) if wl.vortices is not None else None

    t = wl.t0
    # warmup; its last step has every kernel group timed, to find the dominant
    # one (the first step carries first-launch costs)
    for k in range(warmup):
        if k == warmup - 1:
            torch.cuda.synchronize()
            ctx.vrm_timing(True)
        ctx.vrm_step(cloud, P, vt, t)
        t += wl.dt
    torch.cuda.synchronize()
    warm_timers, _ = ctx.vrm_read_timing()
    ctx.vrm_timing(False)
    dom = dominant_group(warm_timers, wl.q)
    c0 = ctx.vrm_read_counters()
    n0 = cloud.n
    # timed region: HIP events around the dominant group's launches only (the
    # other launches carry no events)
    ctx.vrm_timing_groups([dom])
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
    # breakdown over every group, from a few further steps (outside the timed region)
    ctx.vrm_timing(True)
    nb = min(steps, 10)
    for _ in range(nb):
        ctx.vrm_step(cloud, P, vt, t)
        t += wl.dt
    torch.cuda.synchronize()
    breakdown, _ = ctx.vrm_read_timing()
    ctx.vrm_timing(False)
    return dict(elapsed=elapsed, counters=d, timers=timers, timer_overflow=overflow, n_start=n0, n_end=cloud.n,
                final=c1, dominant=dom, breakdown=breakdown, breakdown_steps=nb)


def breakdown(res):
    return {k: round(v[0] / max(1, res["breakdown_steps"]), 4) for k, v in res["breakdown"].items() if v[1] > 0}


def dominant_group(timers, q):
    """The kernel group with the largest time (insertion, with its host synchronisations, excluded)."""
    cand = {k: v for k, v in timers.items() if k != "insert" and v[1] > 0}
    if not cand:
        return "lp_small" if q == 2 else "lp_full"
    return max(cand, key=lambda k: cand[k][0])


# training geometry of the warm-start network for each workload (other seeds, same generator)
TRAINING = {
    "lamb_oseen_h0.01_q2": dict(kind="lamb_oseen", h=0.01, q=2),
    "lamb_oseen_h0.01_q3": dict(kind="lamb_oseen", h=0.01, q=3),
    "vortices64_h0.005": dict(kind="vortices", h=0.02, q=2),
    "vortices256_h0.004_q3": dict(kind="vortices_dense", h=0.02, q=3),
}


def train_network(name, seeds, epochs):
    """Warm-start network trained on the GPU from the plain solver's stencils of
    `seeds` snapshots of the workload's generator (seeds 1000+, never the timed one)."""
    import torch
    import paper_1508_06379_amd as vrm
    import paper_1508_06379_amd.learned as L
    spec = TRAINING[name]
    t0 = time.perf_counter()
    X, Y = L.collect(lambda s: workloads.training_snapshot(1000 + s, h=spec["h"], q=spec["q"], kind=spec["kind"]),
                     range(seeds))
    t1 = time.perf_counter()
    ctx = vrm.Context(64)
    # 9-row bases learn better with a light fraction term and a higher rate
    wf, lr = (1.0, 1e-3) if spec["q"] == 2 else (0.1, 3e-3)
    if spec["q"] == 3:
        epochs = max(epochs, 20)
    hist = L.train(ctx, X, Y, epochs=epochs, batch=4096, lr=lr, weight_decay=1e-4, frac_weight=wf, seed=spec["q"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    acc = L.basis_accuracy(ctx, X[:200000], Y[:200000], spec["q"])
    theta = torch.zeros(vrm.MLP_PARAMS, device="cuda")
    ctx.vrm_mlp_read(theta)
    info = {"rows": int(X.shape[0]), "snapshots": seeds, "generator": spec, "epochs": epochs, "lr": lr,
            "fraction_loss_weight": wf,
            "loss_first_last": [round(hist[0], 4), round(hist[-1], 4)], "train_basis_accuracy": round(acc, 4),
            "collect_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2)}
    return theta, info


def kernel_sources_sha():
    """SHA-256 of the HIP sources: stored byte counts are used only for the build they were taken on."""
    import hashlib
    d = os.path.join(ROOT, "paper_1508_06379_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, group):
    """HBM bytes per launch of `group` from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    summarised under profiles/ (copy-calibrated), or None if the kernels changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(workload)
    if not rec or rec.get("group") != group or rec.get("sources_sha256") != kernel_sources_sha():
        return None
    return rec["bytes_per_launch"]


def roofline(wl, res, workload):
    """Roofline of the dominant kernel group, timed by HIP events in the timed region."""
    dom = res["dominant"]
    ms, launches = res["timers"][dom]
    avg_s = ms / 1e3 / launches
    c = res["counters"]
    m = 5 if wl.q == 2 else 9
    if dom in ("lp_small", "lp_full"):
        # revised simplex with an explicit m x m inverse, per pivot: reduced costs of
        # the k columns (2 m k), prices, entering column and rank-one update of the
        # inverse (2 m^2 each); k = 8 (small) or the mean complete-neighbourhood size
        nlp = c["n_small"] if dom == "lp_small" else max(1, c["n_full"])
        k = 8.0 if dom == "lp_small" else c["full_cols"] / max(1, c["n_full"])
        flops = c["pivots"] * (2.0 * m * k + 6.0 * m * m)
        per_launch = flops / launches
        ach = per_launch / avg_s / 1e12
        return {"kernel": dom, "bound": "alu", "achieved": ach, "peak": PEAK_FP32_NONPACKED_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_NONPACKED_TFLOPS, "traffic": measured_traffic(workload, dom),
                "avg_launch_ms": avg_s * 1e3, "launches": launches,
                "flop_model": f"pivots x (2 m k + 6 m^2), m={m}, k={k:.2f}, {c['pivots'] / max(1, nlp):.2f} pivots/LP"}
    npart = 0.5 * (res["n_start"] + res["n_end"])
    per_launch = BYTES_PER_PARTICLE[dom] * npart
    ach = per_launch / avg_s / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": measured_traffic(workload, dom), "avg_launch_ms": avg_s * 1e3, "launches": launches}


def cpu_baseline(wl, budget_s=15.0, max_steps=10000):
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


def run_removal(reps=3, oracle_too=True):
    """Particle removal (Sec. 6, outlook) on the close-pair cloud over [-4, 4]^2 at
    h = 0.005: 2.56 M jittered sites plus 5 % planted particles closer than r h
    (2.69 M).  Wall time of vrm_remove_particles (it synchronises) on a fresh copy
    of the cloud per call, median of `reps` after one untimed call; the oracle
    does the same removal once on the host for comparison."""
    import torch
    import paper_1508_06379_amd as vrm
    wl = workloads.config_close_pairs(h=0.005, q=2, lo=-4.0, hi=4.0, seed=21)
    P = vrm.params_of(wl)
    ctx = vrm.Context(wl.n + 1024)
    times = []
    for rep in range(reps + 1):
        cloud = vrm.Cloud(wl.x, wl.y, wl.gamma, capacity=wl.n + 1024)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nr, nc = ctx.vrm_remove_particles(cloud, P)
        torch.cuda.synchronize()
        if rep:
            times.append(time.perf_counter() - t0)
        del cloud
    el = float(np.median(times))
    out = {"workload": f"close_pairs_h0.005_[-4,4]^2", "n": wl.n, "candidates": nc, "removed": nr,
           "ms": el * 1e3, "removed_per_s": nr / el, "particles_per_s": wl.n / el}
    if oracle_too:
        import oracle
        x, y, g = (a.astype(np.float64) for a in (wl.x, wl.y, wl.gamma))
        t0 = time.perf_counter()
        ref = oracle.remove(x, y, g, wl.ids, oracle.params_of(wl))
        ot = time.perf_counter() - t0
        out["oracle"] = {"s": ot, "removed": int(ref.removed_ids.size), "cores": 1}
    log(f"removal: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lamb_oseen_h0.01_q2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--solver", default="all", choices=["all", "both", "plain", "learned", "previous", "phase1"],
                    help="plain batched solver, learned warm start, previous-basis warm start, the first "
                         "feasible vertex (phase I only); both = plain + learned, all = the four on the same "
                         "workload")
    ap.add_argument("--train-snapshots", type=int, default=30)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--no-removal", action="store_true", help="skip the particle-removal measurement")
    ap.add_argument("--removal-only", action="store_true",
                    help="only the particle-removal measurement (one JSON object)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also copy a 256 MiB buffer five times (reference kernel for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the redistribution path has no multi-GPU mode "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    if args.removal_only:
        print(json.dumps({"removal": run_removal(oracle_too=not args.no_cpu_baseline)}), flush=True)
        return
    wl = WORKLOADS[args.workload]()
    log(f"workload {args.workload}: N={wl.n} h={wl.h} q={wl.q} dt={wl.dt}")
    from paper_1508_06379_amd import autotune
    tuning = autotune.load(args.workload)   # launch shapes chosen by the autotuner, if any
    log(f"tuning: {tuning}")
    runs = {}
    if args.solver in ("all", "both", "plain"):
        runs["plain"] = run_gpu(wl, args.steps, args.warmup, tuning=tuning)
    train_info = None
    if args.solver in ("all", "previous"):
        runs["previous"] = run_gpu(wl, args.steps, args.warmup, warm_mode=2, tuning=tuning)
    if args.solver in ("all", "phase1"):
        runs["phase1"] = run_gpu(wl, args.steps, args.warmup, tuning=tuning, lp_objective=1)
    if args.solver in ("all", "both", "learned"):
        theta, train_info = train_network(args.workload, args.train_snapshots, args.epochs)
        log(f"network: {train_info}")
        runs["learned"] = run_gpu(wl, args.steps, args.warmup, theta=theta, tuning=tuning)
    if args.calibrate_copy:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 copies of {src.numel() * 4} bytes")
    main_solver = next(k for k in ("plain", "learned", "previous", "phase1") if k in runs)
    res = runs[main_solver]
    c = res["counters"]
    value = c["redistributions"] / res["elapsed"]
    for k, r in runs.items():
        log(f"{k}: elapsed {r['elapsed']:.4f} s, counters {r['counters']}, timed group {r['dominant']} "
            f"{r['timers'][r['dominant']]}, breakdown {r['breakdown']}")
    rl = roofline(wl, res, args.workload)
    line = {
        "metric": "particle redistributions/s (learned warm start vs plain), FP32, moments <= 1e-6",
        "value": value, "unit": "redistributions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["elapsed"] * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "h": wl.h, "q": wl.q, "n_start": res["n_start"],
                   "n_end": res["n_end"], "dt": wl.dt, "solver": main_solver},
        "roofline": rl,
        "tuning": tuning,
        # kernel time per step and group, from steps after the timed region with every group timed
        "breakdown_ms_per_step": breakdown(res),
        "lp": {"small": c["n_small"], "full": c["n_full"], "infeasible": c["n_infeasible"],
               "uncertified": c["n_uncertified"], "pivots": c["pivots"]},
    }
    if "previous" in runs and main_solver != "previous":
        r = runs["previous"]
        cp = r["counters"]
        pv = cp["redistributions"] / r["elapsed"]
        nlp = max(1, cp["warm_hit"] + cp["warm_phase2"] + cp["warm_cold"])
        line["previous_basis"] = {
            "value": pv, "ms_per_step": r["elapsed"] * 1e3 / args.steps, "vs_plain": pv / value,
            "warm_start": {"optimal_from_previous": cp["warm_hit"] / nlp, "phase2_from_previous": cp["warm_phase2"] / nlp,
                           "left_for_cold_solve": cp["warm_cold"] / nlp},
            "pivots": cp["pivots"], "uncertified": cp["n_uncertified"],
            "breakdown_ms_per_step": breakdown(r),
        }
    if "phase1" in runs and main_solver != "phase1":
        r = runs["phase1"]
        cp = r["counters"]
        pv = cp["redistributions"] / r["elapsed"]
        line["phase1_only"] = {
            "value": pv, "ms_per_step": r["elapsed"] * 1e3 / args.steps, "vs_plain": pv / value,
            "pivots": cp["pivots"], "pivots_per_lp": cp["pivots"] / max(1, cp["n_small"] + cp["n_full"]),
            "uncertified": cp["n_uncertified"], "breakdown_ms_per_step": breakdown(r),
            "note": "first feasible vertex (the paper's phase I); stencils differ from the canonical ones",
        }
    if "learned" in runs:
        r = runs["learned"]
        cl = r["counters"]
        lv = cl["redistributions"] / r["elapsed"]
        nlp = max(1, cl["warm_hit"] + cl["warm_phase2"] + cl["warm_cold"])
        line["learned"] = {
            "value": lv, "ms_per_step": r["elapsed"] * 1e3 / args.steps,
            "vs_plain": lv / value if main_solver == "plain" else None,
            "warm_start": {"optimal_from_prediction": cl["warm_hit"] / nlp, "phase2_from_prediction": cl["warm_phase2"] / nlp,
                           "left_for_cold_solve": cl["warm_cold"] / nlp},
            "pivots": cl["pivots"], "uncertified": cl["n_uncertified"],
            "breakdown_ms_per_step": breakdown(r),
            "network": train_info,
        }
    if not args.no_removal:
        line["removal"] = run_removal(oracle_too=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, budget_s=args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
