"""Timing data and training for the learned planner's cost model.

The evaluator generates its own training data: ``timing_sweep`` plans plain
products C = op(A) op(B) of the given shapes and runs the autotuner on each
with the context's timing log open, so every tile / split-K configuration it
times becomes one record (the autotune runs of other workloads can share the
same log). ``dataset`` turns records into the model's features and
log-microsecond targets; ``train`` fits a model on the GPU with the library's
own kernels.
"""
from __future__ import annotations

import json
import math

import numpy as np

from . import hexla as hx


def log_uniform_shapes(seed: int, count: int, lo: int = 16, hi: int = 8192,
                       transposes: bool = True) -> list:
    """(m, n, k, ta, tb) with m, n, k log-uniform in [lo, hi]."""
    g = np.random.default_rng(seed)
    d = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), (count, 3)))).astype(np.int64)
    t = g.integers(0, 2, (count, 2)) if transposes else np.zeros((count, 2), np.int64)
    return [(int(a), int(b), int(c), int(x), int(y)) for (a, b, c), (x, y) in zip(d, t)]


def timing_sweep(ctx, shapes, log_path, dtype=None, reps=2, device="cuda"):
    """Autotunes C = op(A) op(B) for every (m, n, k, ta, tb) with the timing
    log at log_path (appended). Inputs are N(0, 1)."""
    import torch
    dtype = dtype or torch.float32
    ctx.timing_log(log_path)
    try:
        for m, n, k, ta, tb in shapes:
            a = torch.randn((m, k) if ta else (k, m), dtype=dtype, device=device)
            b = torch.randn((k, n) if tb else (n, k), dtype=dtype, device=device)
            # a row-major (r, c) tensor binds as the transpose of its column-major view
            ea = ctx.leaf(a) if ta else hx.trans(ctx.leaf(a))
            eb = ctx.leaf(b) if tb else hx.trans(ctx.leaf(b))
            p = ctx.plan(ea @ eb)
            out, ws = p.output(device), p.workspace(device)
            p.autotune(out, ws, reps=reps)
            ctx.clear()
            del p, out, ws, a, b
    finally:
        ctx.timing_log(None)


def read_log(path) -> list:
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def dataset(records):
    """Features [N, 32] and targets log(us) [N] as float32 numpy arrays."""
    x = np.stack([hx.product_features(r["dtype"], r["precision"], r["mode"], r["ta"], r["tb"],
                                      r["m"], r["n"], r["k"], r["tile"], r["split"])
                  for r in records]).astype(np.float32)
    y = np.log(np.array([max(r["us"], 1e-3) for r in records], dtype=np.float64)).astype(np.float32)
    return x, y


def train(ctx, x, y, epochs=200, batch=256, lr=1e-3, seed=1, model_seed=0, device="cuda"):
    """Fits a new model on (x, y); returns (model, final standardised MSE)."""
    import torch
    xt = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(device)
    yt = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(device)
    m = hx.Model.create(ctx, model_seed)
    loss = m.train(xt, yt, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return m, loss
