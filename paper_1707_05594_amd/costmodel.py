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

from . import (COMPUTE, DTYPES, MLP, TK_FEATURES, TK_TILE_COUNT, TuckerError, mlp_param_count,
               pair_features, time_ttm, time_ttm_pair, ttm_features, ttm_tree_plan)


def node_views(L, K, plan, rank, tdtype="f32", compute="fp32"):
    """(A, L, B, K, in_dtype, compute) of every internal node of tree `rank`,
    as the engine runs it (from the library: per-node storage types and
    compute modes of hooi_init)."""
    return [(v["A"], v["L"], v["B"], v["K"], v["in_dtype"], v["compute"])
            for v in plan.node_views(rank, tdtype, compute)]


def candidate_views(L, K, topk=8, tdtype="f32", compute="fp32"):
    """Distinct node views over the planner's `topk` best trees."""
    plan = ttm_tree_plan(L, K, "dp", topk=topk)
    seen = {}
    for r in range(plan.count):
        for v in node_views(L, K, plan, r, tdtype, compute):
            seen[v] = True
    return list(seen)


def root_pair_view(L, K, plan, rank):
    """(A, Lp, M, Lq, B, Kp, Kq) of tree `rank`'s two root children, or None."""
    return plan.root_pair(rank)[0]


def candidate_pairs(L, K, topk=8, trailing=True):
    """Distinct root-pair views of the two trailing modes (the only pairs the
    engine fuses: the slab pair kernel) over the planner's `topk` best trees,
    plus (trailing=True) that pair whatever tree holds it (more training
    data for the kernel)."""
    plan = ttm_tree_plan(L, K, "dp", topk=topk)
    seen = {}
    for r in range(plan.count):
        v = root_pair_view(L, K, plan, r)
        if v is not None and v[2] == 1 and v[4] == 1:
            seen[v] = True
    if trailing and len(L) >= 3:
        N = len(L)
        seen[(int(np.prod(L[:N - 2], dtype=np.int64)), L[N - 2], 1, L[N - 1], 1, K[N - 2],
              K[N - 1])] = True
    return list(seen)


def random_pair_views(count, seed, min_elems=int(2e7), max_elems=int(3e9)):
    """Seeded root-pair views (A, Lp, 1, Lq, 1, Kp, Kq) of two trailing modes
    in the slab pair kernel's domain (Lp, Lq multiples of 4 with Lp Lq <= 2048,
    ranks up to 8), with |T| log-uniform in [min_elems, max_elems]: the
    root level is where a tree's time goes, so its views are large."""
    g = np.random.Generator(np.random.Philox(np.random.SeedSequence([17070559, 11, seed])))
    out = []
    while len(out) < count:
        Lp, Lq = 4 * int(g.integers(2, 25)), 4 * int(g.integers(2, 25))
        if Lp * Lq > 2048:
            continue
        E = float(np.exp(g.uniform(np.log(min_elems), np.log(max_elems))))
        A = max(4096, int(E / (Lp * Lq)))
        Kp = int(g.integers(1, min(8, Lp) + 1))
        Kq = int(g.integers(1, min(8, Lq) + 1))
        out.append((A, Lp, 1, Lq, 1, Kp, Kq))
    return out


def pair_node_views(pairs, tdtype="f32", compute="fp32"):
    """The two separate root TTMs of each pair view: T as [A, Lp, M Lq B]
    and as [A Lp M, Lq, B]."""
    out = []
    for A, Lp, M, Lq, B, Kp, Kq in pairs:
        out.append((A, Lp, M * Lq * B, Kp, tdtype, compute))
        out.append((A * Lp * M, Lq, B, Kq, tdtype, compute))
    return out


def measure_pairs(pairs, reps=10, device="cuda:0"):
    """Time the fused root pair for every view a pair kernel takes (FP32);
    returns features X, log-ms y and rows (view, ms)."""
    import torch
    dev = torch.device(device)
    X, y, rows = [], [], []
    if not pairs:
        return np.zeros((0, TK_FEATURES), np.float32), np.zeros(0, np.float32), rows
    cap_in = max(A * Lp * M * Lq * B for A, Lp, M, Lq, B, _, _ in pairs)
    cap_p = max(A * Kp * M * Lq * B for A, Lp, M, Lq, B, Kp, _ in pairs)
    cap_q = max(A * Lp * M * Kq * B for A, Lp, M, Lq, B, _, Kq in pairs)
    cap_f = max(max(Lp * Kp, Lq * Kq) for _, Lp, _, Lq, _, Kp, Kq in pairs)
    inp = torch.full((cap_in,), 0.5, dtype=torch.float32, device=dev)
    op = torch.empty((cap_p,), dtype=torch.float32, device=dev)
    oq = torch.empty((cap_q,), dtype=torch.float32, device=dev)
    F = torch.full((cap_f,), 0.25, dtype=torch.float32, device=dev)
    for v in pairs:
        A, Lp, M, Lq, B, Kp, Kq = v
        try:
            ms = time_ttm_pair(inp, A, Lp, M, Lq, B, F, Kp, F, Kq, op, oq, reps=reps)
        except TuckerError:
            continue  # no pair kernel takes this shape
        X.append(pair_features(A, Lp, M, Lq, B, Kp, Kq))
        y.append(math.log(max(ms, 1e-4)))
        rows.append((v, ms))
    del inp, op, oq, F
    return (np.array(X, dtype=np.float32).reshape(-1, TK_FEATURES),
            np.array(y, dtype=np.float32), rows)


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


def measure(views, reps=5, tiles=range(TK_TILE_COUNT), device="cuda:0"):
    """Time every (view, tile) for views (A, L, B, K, in_dtype, compute) at
    their own compute mode (FP32 or reduced; FP64 views are skipped: the
    tree kernels differ there only by shape); returns features X
    (n x TK_FEATURES), log-ms y and rows."""
    import torch
    dev = torch.device(device)
    views = [v for v in views if v[5] != "fp64"]
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
    cap_in = max(A * L * B for A, L, B, _, _, _ in views)
    cap_out = max(A * K * B for A, _, B, K, _, _ in views)
    cap_f = max(L * K for _, L, _, K, _, _ in views)
    bufs = {}
    for dt in sorted({v[4] for v in views}):
        bufs[dt] = torch.full((cap_in,), 0.5, dtype=tdt[dt], device=dev)
    F = torch.full((cap_f,), 0.25, dtype=torch.float32, device=dev)
    out = torch.empty((cap_out,), dtype=torch.float32, device=dev)
    X, y, rows = [], [], []
    for (A, L, B, K, dt, comp) in views:
        for t in tiles:
            ms = time_ttm(bufs[dt], A, L, B, F, K, out, compute=comp, tile=t, reps=reps)
            X.append(ttm_features(A, L, B, K, dt, comp, t))
            y.append(math.log(max(ms, 1e-4)))
            rows.append((A, L, B, K, dt, comp, t, ms))
    del bufs, F, out
    return np.array(X, dtype=np.float32), np.array(y, dtype=np.float32), rows


def training_set(n_shapes=10, n_pairs=48, seed=1, topk=8):
    """Timed training rows: the nodes of the `topk` best trees of `n_shapes`
    random tensors, their root pairs a pair kernel takes, and `n_pairs` random
    trailing-pair views with their two separate root TTMs.  Returns
    (X, y, node_rows, pair_rows)."""
    views, pairs = [], []
    for Ls, Ks in random_shapes(n_shapes, seed=seed):
        views += candidate_views(Ls, Ks, topk=topk)
        pairs += candidate_pairs(Ls, Ks, topk=topk)
    rp = random_pair_views(n_pairs, seed=seed)
    pairs += rp
    views += pair_node_views(rp)
    views = list(dict.fromkeys(views))
    pairs = list(dict.fromkeys(pairs))
    X, y, rows = measure(views)
    Xp, yp, prow = measure_pairs(pairs)
    return np.vstack([X, Xp]), np.concatenate([y, yp]), rows, prow


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
    model.fit_norm(X)
    # the output bias starts at the mean target, so training starts near the data
    p = model.params()
    p[-1] = float(np.mean(y))
    model.set_params(p)
    losses = model.train(X, y, steps, lr)
    return model, losses
