"""Training driver of the learned warm start (marshalling around the C ABI).

Data: the plain GPU solver's own optimal stencils on jittered Lamb-Oseen
clouds (the generator of the h = 0.01 workload, other seeds); every LP gives
one row: its column offsets (network input) and the indicators and values of
its non-zero fractions (targets).  Training: mini-batch AdamW steps, each one
forward + backward pass of the BF16 matrix-core kernels in libvrm.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import MLP_IN, MLP_OUT, MLP_PARAMS, Cloud, Context, params_of

SHAPES = [(MLP_IN, 128), (128,), (128, 128), (128,), (128, MLP_OUT), (MLP_OUT,)]


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; FP32 vector in the ABI layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        parts.append(rng.normal(0.0, math.sqrt(2.0 / s[0]), s).ravel() if len(s) == 2 else np.zeros(s[0]))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == MLP_PARAMS
    return theta


def collect(workload_fn, seeds, max_rows_per_cloud=65536, capacity=None, log=None):
    """Rows (x BF16 as int16, y FP32) from the plain solver on each seed's cloud, on the GPU."""
    import torch
    xs, ys = [], []
    ctx = None
    for s in seeds:
        wl = workload_fn(s)
        cap = capacity or 4 * wl.n + 1024
        if ctx is None or ctx.capacity < cap:
            ctx = Context(cap)
        cloud = Cloud(wl.x, wl.y, wl.gamma, capacity=cap)
        P = params_of(wl)
        ctx.vrm_insert_particles(cloud, P)
        x = torch.empty((max_rows_per_cloud, MLP_IN), dtype=torch.int16, device="cuda")
        y = torch.empty((max_rows_per_cloud, MLP_OUT), dtype=torch.float32, device="cuda")
        rows = ctx.vrm_collect_training(cloud, P, x, y)
        xs.append(x[:rows].clone())
        ys.append(y[:rows].clone())
        if log:
            log(f"collect seed {s}: {rows} rows")
    return torch.cat(xs), torch.cat(ys)


def train(ctx: Context, X, Y, epochs=3, batch=4096, lr=1e-3, weight_decay=1e-4, frac_weight=1.0, seed=0,
          theta0=None, log=None):
    """AdamW on the masked BCE + MSE loss; returns the per-epoch mean losses."""
    import torch
    if theta0 is None:
        theta0 = init_params(seed)
    ctx.vrm_mlp_load(torch.as_tensor(theta0, device="cuda"))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    n = X.shape[0]
    history = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = torch.randperm(n, device="cuda", generator=gen)
        tot = torch.zeros(1, dtype=torch.float64, device="cuda")
        nb = 0
        for b0 in range(0, n - batch + 1, batch):
            idx = order[b0:b0 + batch]
            xb = X.index_select(0, idx).contiguous()
            yb = Y.index_select(0, idx).contiguous()
            ctx.vrm_mlp_train_step(xb, yb, batch, lr, weight_decay, frac_weight, loss)
            tot += loss
            nb += 1
        history.append(float(tot.item()) / max(1, nb))
        if log:
            log(f"epoch {ep}: loss {history[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
    return history


def basis_accuracy(ctx: Context, X, Y, q: int):
    """Fraction of rows whose top-m logits are exactly the optimal stencil's support
    (supports smaller than m count when they are contained in the top m)."""
    import torch
    m = 5 if q == 2 else 9
    pred = torch.empty((X.shape[0], MLP_OUT), dtype=torch.float32, device="cuda")
    ctx.vrm_mlp_infer(X, X.shape[0], pred)
    mask = X[:, 64:96] != 0
    logits = pred[:, :32].masked_fill(~mask, -1e30)
    top = torch.topk(logits, m, dim=1).indices
    chosen = torch.zeros_like(mask)
    chosen.scatter_(1, top, True)
    support = Y[:, :32] > 0.5
    ok = (support & ~chosen).sum(1) == 0
    return float(ok.float().mean().item())
