"""Throughput of the vorticity redistribution hot path on one MI355X.

A step is one SSP-RK3 step of the whole path: reduced-operator selection,
insertion and reordering (once per step), then for each of the three stages
the cell list, the neighbourhoods, the moment LPs (small ones, then the
complete neighbourhoods: column lists, size bins, LPs), the scatter of
nu sum_j f_ji Gamma_j and the stage combination.  The metric counts the
stencils found and applied per second.

Default workload: 256 vortices on [-8, 8]^2 at h = 0.004 (16.0 M particles,
q = 3), the largest configuration on one GPU.  Timing, per solver:
  * the timed region: `--steps` whole steps replayed from the step's HIP graph,
    wall time between two device synchronisations, no events;
  * a breakdown pass (3 steps, every kernel group timed with HIP events, direct
    launches) that names the dominant group;
  * a roofline pass (`--roofline-steps` steps, only the dominant group timed with
    HIP events on the context's stream) for its average launch duration.

Prints ONE JSON line on stdout (everything else goes to stderr).
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# MI355X published peaks: HBM 8 TB/s; FP32 vector 157.3 TFLOP/s (packed FP32,
# which this library never emits: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA)
# x 2.4 GHz = 78.6 TFLOP/s without it); BF16 dense matrix cores 2.5 PFLOP/s
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = 78.6

# algorithmic bytes per particle of the memory-bound kernel groups
BYTES_PER_PARTICLE = {
    "cells": 36.0,     # read x, y, id; write cell, rank, perm and x, y, id in slot order
    "nbhd": 42.0,      # own x, y, id, diffused; small neighbourhood (8 x 4 B) and a queue entry
    "combine": 40.0,   # read x0, y0, g0, x, y, g, u, v, acc; write x, y, g, acc (heat: no x/u traffic)
    "select": 20.0,    # four passes over |Gamma| and the mask
    "full_cols": 44.0,  # own x, y; the record row (37.5 x 4 B would be the columns: 150 B) -- see DESIGN
}

WORKLOADS = workloads.BENCH
DEFAULT_WORKLOAD = "vortices256_h0.004_q3"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(wl, steps, warmup, theta=None, warm_mode=0, tuning=None, lp_objective=0, roofline_steps=10,
            profile=True):
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
    for _ in range(warmup):
        ctx.vrm_step(cloud, P, vt, t)
        t += wl.dt
    torch.cuda.synchronize()
    c0 = ctx.vrm_read_counters()
    n0 = cloud.n
    # the timed region: graph replays, no events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.vrm_step(cloud, P, vt, t)
        t += wl.dt
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    c1 = ctx.vrm_read_counters()
    keys = ("redistributions", "pivots", "n_small", "n_full", "n_infeasible", "n_uncertified", "full_cols",
            "warm_hit", "warm_phase2", "warm_cold", "graph_replays")
    d = {k: c1[k] - c0[k] for k in keys}
    out = dict(elapsed=elapsed, counters=d, n_start=n0, n_end=cloud.n, final=c1)
    if not profile:
        return out
    # breakdown: every group timed (direct launches) over a few steps
    nb = 3
    ctx.vrm_timing(True)
    for _ in range(nb):
        ctx.vrm_step(cloud, P, vt, t)
        t += wl.dt
    torch.cuda.synchronize()
    bd, _ = ctx.vrm_read_timing()
    ctx.vrm_timing(False)
    dom = dominant_group(bd, wl.q)
    # roofline pass: only the dominant group's launches bracketed by events
    ctx.vrm_timing_groups([dom])
    r0 = ctx.vrm_read_counters()
    for _ in range(roofline_steps):
        ctx.vrm_step(cloud, P, vt, t)
        t += wl.dt
    torch.cuda.synchronize()
    timers, overflow = ctx.vrm_read_timing()
    ctx.vrm_timing(False)
    r1 = ctx.vrm_read_counters()
    rc = {k: r1[k] - r0[k] for k in keys}
    out.update(breakdown=bd, breakdown_steps=nb, dominant=dom, roofline_timers=timers, roofline_counters=rc,
               roofline_steps=roofline_steps, timer_overflow=overflow)
    return out


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
# rows taken from each training cloud (about 10 M solves for the 16 M-particle cloud's network)
ROWS_PER_SNAPSHOT = {"vortices256_h0.004_q3": 1 << 18}
TRAIN_SNAPSHOTS = {"vortices256_h0.004_q3": 100}


def train_network(name, seeds, epochs):
    """Warm-start network trained on the GPU from the plain solver's stencils of
    `seeds` snapshots of the workload's generator (seeds 1000+, never the timed one)."""
    import torch
    import paper_1508_06379_amd as vrm
    import paper_1508_06379_amd.learned as L
    spec = TRAINING[name]
    t0 = time.perf_counter()
    X, Y = L.collect(lambda s: workloads.training_snapshot(1000 + s, h=spec["h"], q=spec["q"], kind=spec["kind"]),
                     range(seeds), max_rows_per_cloud=ROWS_PER_SNAPSHOT.get(name, 65536))
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
    """Roofline of the dominant kernel group: algorithmic work per launch (counters of
    the roofline pass) over the average launch duration (HIP events of that pass)."""
    dom = res["dominant"]
    ms, launches = res["roofline_timers"][dom]
    avg_s = ms / 1e3 / max(1, launches)
    c = res["roofline_counters"]
    m = 5 if wl.q == 2 else 9
    if dom in ("lp_small", "lp_full"):
        # simplex work per pivot: 2 m (k + 1) FLOP (pricing of the k columns and the
        # update of the m x (k + 1) tableau it stands for); k = 8 (small) or the mean
        # complete-neighbourhood size; pivots and k measured by the counters
        nlp = c["n_small"] if dom == "lp_small" else max(1, c["n_full"])
        k = 8.0 if dom == "lp_small" else c["full_cols"] / max(1, c["n_full"])
        flops = c["pivots"] * 2.0 * m * (k + 1.0)
        per_launch = flops / max(1, launches)
        ach = per_launch / avg_s / 1e12
        traffic = measured_traffic(workload, dom)
        return {"kernel": dom, "bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
                "frac_of_nonpacked_peak": ach / PEAK_FP32_NONPACKED_TFLOPS, "traffic": traffic,
                "avg_launch_ms": avg_s * 1e3, "launches": launches, "lps_per_launch": nlp / max(1, launches),
                "flop_model": f"pivots x 2 m (k + 1), m={m}, k={k:.2f}, {c['pivots'] / max(1, nlp):.2f} pivots/LP",
                "timing": "HIP events on the context's stream around every launch of the group, "
                          f"{res['roofline_steps']} steps after the timed region"}
    npart = 0.5 * (res["n_start"] + res["n_end"])
    per_launch = BYTES_PER_PARTICLE[dom] * npart
    ach = per_launch / avg_s / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": measured_traffic(workload, dom), "avg_launch_ms": avg_s * 1e3,
            "launches": launches}


def host_info():
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(wl, name, budget_s=15.0):
    """The FP64 oracle on the host cores: whole SSP-RK3 steps of a bounded sample of
    the same workload (the small clouds from their initial state; the vortex clouds
    on a square window of the same generated cloud, its size chosen for about
    `budget_s` of work), as redistributions per second."""
    import oracle
    oracle.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if wl.n > 200000:
        # a window with about budget_s of LP work: calibrate on a small one
        probe = workloads.c5_window(wl, 0.3)
        t0 = time.perf_counter()
        st = oracle.step(oracle.initial_state(probe), probe)
        rate = (time.perf_counter() - t0) / max(1, probe.n)
        half = float(np.clip(0.3 * np.sqrt(budget_s / max(1e-9, rate * probe.n)), 0.3, 8.0))
        sample = workloads.c5_window(wl, half)
        desc = (f"one SSP-RK3 step (insertion and three stages) of the particles of the same cloud in "
                f"[-{half:.2f}, {half:.2f}]^2 ({sample.n} of {wl.n}; the window's edge adds insertions)")
        steps_max = 1
    else:
        sample = wl
        desc = "the first SSP-RK3 steps of the same workload from its initial state"
        steps_max = 10000
    st = oracle.initial_state(sample)
    red = 0
    steps = 0
    t0 = time.perf_counter()
    while steps < steps_max and (steps == 0 or time.perf_counter() - t0 < budget_s):
        st = oracle.step(st, sample)
        h = st.history[-1]
        red += h.status_counts[0] + h.status_counts[1]
        steps += 1
    el = time.perf_counter() - t0
    return {"value": red / el, "unit": "redistributions/s", "cores": threads, "kind": "oracle",
            "sample": f"{desc}; {steps} step(s), {red} redistributions in {el:.1f} s; LPs and neighbourhoods "
                      f"OpenMP-parallel over {threads} threads, insertion, selection and the apply scatter serial "
                      f"(the apply in a fixed order)",
            "host": host_info()}


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
    out = {"workload": "close_pairs_h0.005_[-4,4]^2", "n": wl.n, "candidates": nc, "removed": nr,
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


def solver_summary(r, steps, value_plain):
    c = r["counters"]
    v = c["redistributions"] / r["elapsed"]
    nlp = max(1, c["warm_hit"] + c["warm_phase2"] + c["warm_cold"])
    out = {"value": v, "ms_per_step": r["elapsed"] * 1e3 / steps,
           "vs_plain": v / value_plain if value_plain else None,
           "pivots": c["pivots"], "pivots_per_lp": c["pivots"] / max(1, c["n_small"] + c["n_full"]),
           "uncertified": c["n_uncertified"], "infeasible": c["n_infeasible"]}
    if c["warm_hit"] + c["warm_phase2"] + c["warm_cold"]:
        out["warm_start"] = {"optimal_from_start": c["warm_hit"] / nlp, "phase2_from_start": c["warm_phase2"] / nlp,
                             "left_for_cold_solve": c["warm_cold"] / nlp}
    if "breakdown" in r:
        out["breakdown_ms_per_step"] = breakdown(r)
    return out


def solver_accuracy(q=3, h=0.02, T=0.16):
    """Accuracy of the stencil solvers on the Lamb-Oseen case (Sec. 5.1): for the
    canonical LP, the first feasible vertex and non-negative least squares, the
    weak error at T against the closed form, the largest moment residual of the
    last stencils (verification kernel, FP64) and the time per step."""
    import torch
    import paper_1508_06379_amd as vrm
    out = {"workload": f"lamb_oseen jittered lattice h={h} q={q}, SSP-RK3 to T={T}"}
    for name, obj in (("canonical", 0), ("phase1_only", 1), ("nnls", 2)):
        wl = workloads.config_jittered(h=h, q=q, seed=2)
        steps = int(round(T / wl.dt))
        cloud = vrm.Cloud(wl.x, wl.y, wl.gamma, capacity=4 * wl.n + 64)
        ctx = vrm.Context(cloud.capacity)
        ctx.vrm_set_lp_objective(obj)
        P = vrm.params_of(wl)
        t = wl.t0
        ctx.vrm_step(cloud, P, None, t)
        t += wl.dt
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps - 1):
            ctx.vrm_step(cloud, P, None, t)
            t += wl.dt
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / max(1, steps - 1)
        x, y, g, _ = cloud.numpy()
        st = vrm.Stencils.alloc(cloud.capacity)
        ctx.vrm_solve_fractions(cloud, P, st)
        rep = torch.zeros(4, dtype=torch.float64, device="cuda")
        ctx.vrm_verify(cloud, P, st, rep)
        torch.cuda.synchronize()
        out[name] = {"weak_error": workloads.lamb_oseen_weak_error(x, y, g, t, wl.nu),
                     "max_moment_residual": float(rep[0]), "ms_per_step": ms, "steps": steps}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--solver", default="all",
                    choices=["all", "both", "plain", "learned", "previous", "phase1", "nnls"],
                    help="plain batched solver, learned warm start, previous-basis warm start, the first "
                         "feasible vertex (phase I only), non-negative least squares; both = plain + learned, "
                         "all = the five on the same workload")
    ap.add_argument("--roofline-steps", type=int, default=5)
    ap.add_argument("--train-snapshots", type=int, default=0, help="training clouds (0: the workload's default)")
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
    t_gen = time.perf_counter()
    wl = WORKLOADS[args.workload]()
    log(f"workload {args.workload}: N={wl.n} h={wl.h} q={wl.q} dt={wl.dt} (generated in "
        f"{time.perf_counter() - t_gen:.1f} s)")
    from paper_1508_06379_amd import autotune
    tuning = autotune.load(args.workload)   # launch shapes chosen by the autotuner, if any
    log(f"tuning: {tuning}")
    runs = {}
    kw = dict(roofline_steps=args.roofline_steps)
    if args.solver in ("all", "both", "plain"):
        runs["plain"] = run_gpu(wl, args.steps, args.warmup, tuning=tuning, **kw)
        log(f"plain: {runs['plain']['elapsed']:.3f} s, {runs['plain']['counters']}")
    train_info = None
    if args.solver in ("all", "previous"):
        runs["previous"] = run_gpu(wl, args.steps, args.warmup, warm_mode=2, tuning=tuning, **kw)
        log(f"previous: {runs['previous']['elapsed']:.3f} s")
    if args.solver in ("all", "phase1"):
        runs["phase1"] = run_gpu(wl, args.steps, args.warmup, tuning=tuning, lp_objective=1, **kw)
        log(f"phase1: {runs['phase1']['elapsed']:.3f} s")
    if args.solver in ("all", "nnls"):
        runs["nnls"] = run_gpu(wl, args.steps, args.warmup, tuning=tuning, lp_objective=2, **kw)
        log(f"nnls: {runs['nnls']['elapsed']:.3f} s")
    if args.solver in ("all", "both", "learned"):
        theta, train_info = train_network(args.workload, args.train_snapshots or TRAIN_SNAPSHOTS.get(args.workload, 30),
                                          args.epochs)
        log(f"network: {train_info}")
        runs["learned"] = run_gpu(wl, args.steps, args.warmup, theta=theta, tuning=tuning, **kw)
        log(f"learned: {runs['learned']['elapsed']:.3f} s")
    if args.calibrate_copy:
        import torch
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 copies of {src.numel() * 4} bytes")
    main_solver = next(k for k in ("plain", "learned", "previous", "phase1", "nnls") if k in runs)
    res = runs[main_solver]
    c = res["counters"]
    value = c["redistributions"] / res["elapsed"]
    for k, r in runs.items():
        log(f"{k}: elapsed {r['elapsed']:.4f} s, counters {r['counters']}, dominant {r.get('dominant')}, "
            f"breakdown {r.get('breakdown')}")
    rl = roofline(wl, res, args.workload)
    line = {
        "metric": "particle redistributions/s (learned warm start vs plain), FP32, moments <= 1e-6",
        "value": value, "unit": "redistributions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["elapsed"] * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "h": wl.h, "q": wl.q, "n_start": res["n_start"],
                   "n_end": res["n_end"], "dt": wl.dt, "solver": main_solver,
                   "timed": "graph-replayed steps, wall time between device synchronisations"},
        "roofline": rl,
        "tuning": tuning,
        # kernel time per step and group, from steps after the timed region with every group timed
        "breakdown_ms_per_step": breakdown(res),
        "lp": {"small": c["n_small"], "full": c["n_full"], "infeasible": c["n_infeasible"],
               "uncertified": c["n_uncertified"], "pivots": c["pivots"],
               "mean_complete_columns": c["full_cols"] / max(1, c["n_full"])},
    }
    names = {"previous": "previous_basis", "phase1": "phase1_only", "nnls": "nnls", "learned": "learned"}
    for k, key in names.items():
        if k in runs and k != main_solver:
            line[key] = solver_summary(runs[k], args.steps, value if main_solver == "plain" else None)
    if "phase1_only" in line:
        line["phase1_only"]["note"] = "first feasible vertex (the paper's phase I); stencils differ from the canonical ones"
    if "nnls" in line:
        line["nnls"]["note"] = ("non-negative least squares (Lawson-Hanson, Sec. 4.1's alternative); pivots "
                                "count the columns freed")
    if "learned" in line:
        line["learned"]["network"] = train_info
    if args.solver == "all":
        line["solver_accuracy"] = solver_accuracy()
    if not args.no_removal:
        line["removal"] = run_removal(oracle_too=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.workload, budget_s=args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
