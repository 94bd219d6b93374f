"""Learned TTM-tree and kernel selection: training data and training.

The planner's dynamic program (Sec. 3.3) ranks trees by multiply-adds
(Sec. 3.1); trees of equal or nearly equal cost can still differ in run time on
the device, because each node's shape decides which TTM kernel runs and how
well it uses the chip.  This module times TTM nodes on the GPU with the
library's own timer (``time_ttm``), trains the library's MLP on the log of
those times (forward, backward and Adam run in libtucker), and hands the model
to ``Plan.learned``, which picks a tree among the planner's k best and a kernel
per node.  Orchestration only: the shapes to time, the seeded initial
parameters and the feature standardisation are chosen here; every number the
model computes is computed on the device.
"""
from __future__ import annotations

import math

import numpy as np

from . import (COMPUTE, DTYPES, MLP, TK_FEATURES, TK_TILE_COUNT, mlp_param_count, time_ttm,
               ttm_features, ttm_tree_plan)


def node_views(L, K, plan, rank, tdtype="f32", compute="fp32"):
    """(A, L, B, K, in_dtype) of every internal node of tree `rank`."""
    out = []
    for nd in plan.nodes(rank):
        if nd["is_leaf"]:
            continue
        n, pre = nd["mode"], nd["pre_mask"]
        dims = [K[j] if (pre >> j) & 1 else L[j] for j in range(len(L))]
        A = int(np.prod(dims[:n], dtype=np.int64))
        B = int(np.prod(dims[n + 1:], dtype=np.int64))
        in_dt = tdtype if nd["parent"] < 0 else ("f64" if compute == "fp64" else "f32")
        out.append((A, dims[n], B, K[n], in_dt))
    return out


def candidate_views(L, K, topk=8, tdtype="f32", compute="fp32"):
    """Distinct node views over the planner's `topk` best trees."""
    plan = ttm_tree_plan(L, K, "dp", topk=topk)
    seen = {}
    for r in range(plan.count):
        for v in node_views(L, K, plan, r, tdtype, compute):
            seen[v] = True
    return list(seen)


def random_shapes(count, seed, max_elems=int(1.6e9)):
    """Seeded random tensor shapes (4 to 6 modes) and ranks for training data."""
    g = np.random.Generator(np.random.Philox(np.random.SeedSequence([17070559, 9, seed])))
    shapes = []
    while len(shapes) < count:
        N = int(g.integers(4, 7))
        L = [int(g.integers(8, 97)) for _ in range(N)]
        if math.prod(L) > max_elems or math.prod(L) < 1e6:
            continue
        K = [max(1, min(l, int(round(l * g.uniform(0.05, 0.3))))) for l in L]
        for n in range(N):
            K[n] = min(K[n], math.prod(K[m] for m in range(N) if m != n))
        shapes.append((tuple(L), tuple(K)))
    return shapes


def measure(views, compute="fp32", reps=3, tiles=range(TK_TILE_COUNT), device="cuda:0"):
    """Time every (view, tile); returns features X (n x TK_FEATURES), log-ms y."""
    import torch
    dev = torch.device(device)
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f64": torch.float64}
    cap_in = max(A * L * B for A, L, B, _, _ in views)
    cap_out = max(A * K * B for A, _, B, K, _ in views)
    cap_f = max(L * K for _, L, _, K, _ in views)
    out_dt = torch.float64 if compute == "fp64" else torch.float32
    bufs = {}
    for dt in sorted({v[4] for v in views}):
        bufs[dt] = torch.full((cap_in,), 0.5, dtype=tdt[dt], device=dev)
    F = torch.full((cap_f,), 0.25, dtype=out_dt, device=dev)
    out = torch.empty((cap_out,), dtype=out_dt, device=dev)
    X, y, rows = [], [], []
    for (A, L, B, K, dt) in views:
        for t in tiles:
            ms = time_ttm(bufs[dt], A, L, B, F, K, out, compute=compute, tile=t, reps=reps)
            X.append(ttm_features(A, L, B, K, dt, compute, t))
            y.append(math.log(max(ms, 1e-4)))
            rows.append((A, L, B, K, dt, t, ms))
    del bufs, F, out
    return np.array(X, dtype=np.float32), np.array(y, dtype=np.float32), rows


def init_params(in_dim, hidden, seed):
    """He-normal weights, zero biases, from a seeded generator."""
    g = np.random.Generator(np.random.Philox(np.random.SeedSequence([17070559, 10, seed])))
    parts = [g.standard_normal((hidden, in_dim)) * math.sqrt(2.0 / in_dim), np.zeros(hidden),
             g.standard_normal((hidden, hidden)) * math.sqrt(2.0 / hidden), np.zeros(hidden),
             g.standard_normal(hidden) * math.sqrt(1.0 / hidden), np.zeros(1)]
    p = np.concatenate([q.reshape(-1) for q in parts]).astype(np.float32)
    assert p.size == mlp_param_count(in_dim, hidden)
    return p


def train(X, y, hidden=32, steps=3000, lr=3e-3, seed=0):
    """A trained MLP (standardised features); returns (model, per-step losses)."""
    X = np.asarray(X, dtype=np.float32)
    model = MLP(TK_FEATURES, hidden, init_params(TK_FEATURES, hidden, seed))
    mu = X.mean(axis=0)
    sigma = X.std(axis=0)
    sigma = np.where(sigma > 1e-6, sigma, 1.0).astype(np.float32)
    model.set_norm(mu, sigma)
    # the output bias starts at the mean target, so training starts near the data
    p = model.params()
    p[-1] = float(np.mean(y))
    model.set_params(p)
    losses = model.train(X, y, steps, lr)
    return model, losses
