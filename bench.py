"""Benchmark: HOOI iterations/s on one MI355X for the dense Tucker hot path.

Workload: planted 200x200x200x200 FP32 tensor, Tucker rank 20 per mode, 1e-3
relative Gaussian noise, HOSVD start, DP-optimal TTM-tree.  One step is one
HOOI invocation (every TTM of the tree, the Grams, the FP64 eigensolver and
the folded core + error); the timed region is hooi_iterate(steps), whose final
direct core chain (the error of the last step) is included.

Prints ONE JSON line.  Extra objects:
  roofline     -- the dominant kernel (the root-level TTMs that read T), timed
                  with HIP events on the library's stream; algorithmic bytes
                  = 4 * (|In| + |Out|) + factor per launch, HBM peak 8 TB/s;
                  traffic = measured HBM bytes per launch from the committed
                  counter summary under profiles/ (null once the kernel
                  sources differ from those the counters were taken with).
  cpu_baseline -- the FP64 oracle (naive per-mode chains, NumPy) timed on the
                  host for a bounded sample: consecutive HOOI invocations of
                  the same tensor until at least 10 s of CPU work.
  bf16_storage_80x80x80x80x80 -- the 80^5 rank-10 tensor stored as BF16, HOOI with FP32,
                  bf16x3 and BF16 TTMs (precision study), FP64 residual errors.
  batch        -- batched HOOI over 512 planted 3- and 4-mode tensors (grouped
                  persistent TTM levels in a replayed HIP graph).
  mixed        -- the same HOOI with T stored as BF16, TTMs in bf16x3 and in
                  BF16 (BF16 MFMA); each run's factors are scored against the
                  FP32 tensor (FP64 explicit residual) beside the FP32 run's.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HOOI iters/sec + TTM GFLOP/s (% MFMA peak), mixed vs FP32 at equal rel. error"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
WORKLOAD = "planted_200x200x200x200_r20_f32"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


COUNTERS = os.path.join(ROOT, "profiles", "ttm_wide_f32_root_200x200x200x200_r20_hbm_counters.txt")
MFMA_COUNTERS = os.path.join(ROOT, "profiles", "ttm_root_200x200x200x200_r20_mfma_counters.txt")


def recorded_value(path, key, kind=float):
    """A figure from a committed rocprofv3 summary (`key: value` line), or None
    when the kernel sources it names have changed since it was taken."""
    import hashlib
    try:
        text = open(path).read().splitlines()
    except OSError:
        return None
    value, digest, files = None, None, []
    for line in text:
        line = line.strip()
        if line.startswith(key + ":"):
            value = kind(line.split(":")[1])
        elif line.startswith("kernel_source_sha256_16:"):
            parts = line.split(":", 1)[1].split()
            digest = parts[0]
            files = [f.strip("()") for f in parts[1:]]
    if value is None or digest is None or not files:
        return None
    h = hashlib.sha256()
    for f in files:
        try:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        except OSError:
            return None
    return value if h.hexdigest()[:16] == digest else None


def recorded_traffic():
    """HBM bytes per root-TTM launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return recorded_value(COUNTERS, "traffic_bytes_per_launch", int)


def root_ttm_roofline(ctx, plan, reps=3, t_bytes=4, kernel="ttm_wide_f32 (root nodes, reads T)",
                      with_traffic=True):
    """Average duration of the root-level TTM launches (HIP events, ctx stream)."""
    nodes = plan.nodes()
    roots = [i for i, n in enumerate(nodes) if n["parent"] < 0 and not n["is_leaf"]]
    times = []
    for _ in range(reps):
        ms = ctx.profile_tree()
        times.extend(ms[i] for i in roots)
    avg_ms = sum(times) / len(times)
    L, K = plan.L, plan.K
    per_launch = []
    for i in roots:
        n = nodes[i]
        per_launch.append(t_bytes * n["in_card"] + 4 * n["out_card"] + 4 * L[n["mode"]] * K[n["mode"]])
    bytes_per_launch = sum(per_launch) / len(per_launch)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    flops = sum(2 * nodes[i]["in_card"] * K[nodes[i]["mode"]] for i in roots) / len(roots)
    tflops = flops / (avg_ms * 1e-3) / 1e12
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=recorded_traffic() if with_traffic else None,
                kernel=kernel, launches=len(times),
                avg_ms=round(avg_ms, 4), bytes_per_launch=int(bytes_per_launch),
                mfma_tflops=round(tflops, 2), mfma_frac_fp32_peak=round(tflops / FP32_MFMA_PEAK_TFLOPS, 4),
                mfma_busy=(recorded_value(MFMA_COUNTERS, "mfma_busy_root_fp32") if with_traffic
                           else None)), ms


def iteration_bytes(plan, t_bytes=4, w_bytes=4):
    """Algorithmic HBM bytes of one tree pass: (launched, minimum).
    launched: every TTM reads its input and writes its output, every Gram reads
    its leaf (each root child streams T);  minimum: T read once, every
    intermediate written once and read once by each of its children."""
    nodes = plan.nodes()
    kids = [0] * len(nodes)
    for n in nodes:
        if n["parent"] >= 0:
            kids[n["parent"]] += 1
    L, K = plan.L, plan.K
    card_T = 1
    for x in L:
        card_T *= x
    launched = 0
    minimum = t_bytes * card_T
    for u, n in enumerate(nodes):
        if n["is_leaf"]:
            launched += w_bytes * n["in_card"]
            continue
        in_b = t_bytes if n["parent"] < 0 else w_bytes
        launched += in_b * n["in_card"] + w_bytes * n["out_card"] + 4 * L[n["mode"]] * K[n["mode"]]
        minimum += w_bytes * n["out_card"] * (1 + kids[u]) + 4 * L[n["mode"]] * K[n["mode"]]
    return launched, minimum


def iteration_roofline(plan, ms_per_step, t_bytes=4):
    launched, minimum = iteration_bytes(plan, t_bytes)
    s = ms_per_step * 1e-3
    return {"launched_bytes": launched, "min_bytes": minimum,
            "frac_launched": round(launched / s / 1e9 / HBM_PEAK_GBS, 4),
            "frac_min": round(minimum / s / 1e9 / HBM_PEAK_GBS, 4),
            "note": "bytes per HOOI invocation over its measured time, against 8 TB/s: "
                    "launched = every kernel's own reads and writes; min = T read once, "
                    "each intermediate written once and read once per child"}


def cpu_baseline(T32, K, F0, min_seconds=10.0, max_invocations=30):
    """Oracle (FP64 NumPy, naive chains): consecutive HOOI invocations of the
    same tensor, from the GPU's HOSVD factors, until at least `min_seconds`
    of CPU work (a bounded sample of the workload)."""
    import numpy as np
    from oracle import hooi as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    T64 = T32.astype(np.float64)
    F = F0
    n = 0
    t0 = time.perf_counter()
    while n < max_invocations and (n == 0 or time.perf_counter() - t0 < min_seconds):
        F, _, _ = O.hooi_step(T64, F, K)
        n += 1
    dt = time.perf_counter() - t0
    del T64
    return dict(value=round(n / dt, 5), unit="HOOI iters/s", cores=int(threads), kind="oracle",
                sample=f"{n} consecutive FP64 HOOI invocations (naive per-mode TTM chains + eigh "
                       "+ core) of the same 200^4 rank-20 tensor, from the GPU's HOSVD factors",
                seconds=round(dt, 2))


def five_mode_bf16_leg(steps, warmup):
    """The five-mode 80^5 tensor stored as BF16 (rank 10, 1e-2 relative noise):
    HOOI iterations/s with FP32, bf16x3 and BF16 TTMs, each run's error by the
    FP64 explicit residual against the stored tensor."""
    import torch

    import paper_1707_05594_amd as tk
    import synth
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    T, info = synth.workload("planted_80x80x80x80x80_r10_bf16")
    K = info["K"]
    Td = torch.from_numpy(T.view("int16")).view(torch.bfloat16).to(dev)
    del T
    torch.cuda.synchronize()
    log(f"80^5: generated 80^5 BF16 in {time.perf_counter() - t0:.1f}s")
    plan = tk.ttm_tree_plan(info["L"], K)
    res = {"workload": "planted 80x80x80x80x80 stored BF16, Tucker rank 10/mode, 1e-2 rel noise, "
                       "HOSVD start, DP-optimal TTM-tree", "tree": plan.string(),
           "tree_macs": plan.cost()}
    F0 = None
    for compute in ("fp32", "bf16x3", "bf16"):
        ctx = tk.hooi_init(Td, K, plan=plan, compute=compute, F0=F0)
        if F0 is None:
            F0 = ctx.factors()
        ctx.iterate(max(1, warmup))
        ctx.set_factors(F0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        errs = ctx.iterate(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / steps
        res[compute] = {"value": round(1.0 / dt, 3), "unit": "HOOI iters/s",
                        "ms_per_step": round(1e3 * dt, 4), "rel_err": errs[-1],
                        "rel_err_explicit": ctx.error_explicit(),
                        "iteration_roofline": iteration_roofline(plan, 1e3 * dt, t_bytes=2)}
        if compute == "fp32":
            res["roofline"], _ = root_ttm_roofline(
                ctx, plan, t_bytes=2, with_traffic=False,
                kernel="ttm_wide_bf16 (FP32 compute on BF16 T, root nodes, read T)")
        log(f"80^5 {compute}: {res[compute]['value']} it/s, error {res[compute]['rel_err_explicit']:.6e}")
        del ctx
    del Td
    torch.cuda.empty_cache()
    return res


def batch_leg(steps, warmup, seq_count=64):
    """Batched HOOI over the uneven 512-tensor batch (3- or 4-mode, L in
    [32, 128], K in [4, 16], 1e-3 relative noise, FP32): iterations/s of the
    whole batch, the tree's algorithmic bytes per iteration and the rate they
    imply, plus the first `seq_count` tensors run one context after another
    against the same tensors as one batch."""
    import numpy as np
    import torch

    import paper_1707_05594_amd as tk
    import synth
    dev = torch.device("cuda:0")
    shapes = synth.batch_shapes(512, cfg=5, seed_idx=0)
    t0 = time.perf_counter()
    devs = []
    elems = 0
    for i, T in synth.batch_tensors(shapes, noise=1e-3, dtype="f32", cfg=5):
        devs.append(torch.from_numpy(T).to(dev))
        elems += T.size
        del T
    torch.cuda.synchronize()
    log(f"batch: generated and uploaded {len(shapes)} tensors ({elems:.3e} elements) in "
        f"{time.perf_counter() - t0:.1f}s")
    ranks = [K for _, K in shapes]
    b = tk.Batch(devs, ranks)
    bpc, tune_ms = b.tune()
    st = b.stats()
    F0 = b.factors()
    if warmup > 0:
        b.iterate(warmup)
    b.set_factors(F0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    errs = b.iterate(steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / steps
    cur = b.error()
    # the same batch stored as BF16 (FP32 compute: exact products of BF16 data)
    devs_b = [d.to(torch.bfloat16) for d in devs]
    bb = tk.Batch(devs_b, ranks)
    bb.tune()
    Fb0 = bb.factors()
    if warmup > 0:
        bb.iterate(warmup)
    bb.set_factors(Fb0)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    bb.iterate(steps)
    torch.cuda.synchronize()
    dt_bf = (time.perf_counter() - t4) / steps
    cur_b = bb.error()
    stb = bb.stats()
    bf16 = {"storage": "bf16", "value": round(1.0 / dt_bf, 3), "unit": "batch HOOI iters/s",
            "ms_per_step": round(1e3 * dt_bf, 4), "tree_bytes": stb["tree_bytes"],
            "tree_GBps_at_step_time": round(stb["tree_bytes"] / dt_bf / 1e9, 1),
            "frac_hbm_peak": round(stb["tree_bytes"] / dt_bf / 1e9 / HBM_PEAK_GBS, 4),
            "rel_err_median": float(np.median(cur_b)), "rel_err_max": float(np.max(cur_b))}
    log(f"batch bf16 storage: {bf16['value']} it/s ({bf16['ms_per_step']} ms)")
    del bb, devs_b
    # the same first seq_count tensors: one context each, one after another
    sub = list(range(seq_count))
    bs = tk.Batch([devs[i] for i in sub], [ranks[i] for i in sub])
    bs.tune()
    bs.iterate(1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    bs.iterate(steps)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t2) / steps
    # one live context at a time (each holds its own streams and hardware
    # queues); only the iterations are timed
    t_seq = 0.0
    for i in sub:
        c = tk.hooi_init(devs[i], ranks[i], compute="fp32")
        c.iterate(1)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        c.iterate(steps)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t3
        del c
    dt_s = t_seq / steps
    res = {"workload": "512 planted tensors, 3- or 4-mode, L in [32,128], K in [4,16], 1e-3 rel "
                       "noise, FP32, HOSVD start, DP tree each",
           "elements": int(elems), "value": round(1.0 / dt, 3), "unit": "batch HOOI iters/s",
           "ms_per_step": round(1e3 * dt, 4), "tree_macs": st["tree_macs"],
           "tree_bytes": st["tree_bytes"], "levels": st["levels"], "ttm_items": st["ttm_items"],
           "tree_GBps_at_step_time": round(st["tree_bytes"] / dt / 1e9, 1),
           "frac_hbm_peak": round(st["tree_bytes"] / dt / 1e9 / HBM_PEAK_GBS, 4),
           "tuned_blocks_per_cu": bpc, "tune_pass_ms": [round(float(x), 4) for x in tune_ms[:4]],
           "tune_other_row_body_ms": round(float(tune_ms[4]), 4),
           "rel_err_median": float(np.median(cur)), "rel_err_max": float(np.max(cur)),
           "first_%d" % seq_count: {"batched_ms_per_step": round(1e3 * dt_b, 4),
                                    "one_context_each_ms_per_step": round(1e3 * dt_s, 4),
                                    "speedup": round(dt_s / dt_b, 2)},
           "bf16_storage": bf16}
    log(f"batch: {res['value']} it/s ({res['ms_per_step']} ms), tree {st['tree_bytes']/1e9:.1f} GB "
        f"-> {res['tree_GBps_at_step_time']} GB/s; first {seq_count}: batched {1e3*dt_b:.2f} ms vs "
        f"one context each {1e3*dt_s:.2f} ms")
    del b, bs, devs
    torch.cuda.empty_cache()
    return res


def six_mode_leg(steps, warmup):
    """The six-mode 64x48x40x32x24x16 FP32 tensor (ranks 8,8,6,6,4,4, decaying
    core, 1e-3 relative noise): the plain DP tree (separate root TTMs,
    automatic kernels) against the learned choice among the DP's 8 best trees
    and their kernels (the MLP trained on node and root-pair timings of random
    shapes), which may run the two root children as one pass over T.
    HOOI iterations/s of both at their explicit errors; the roofline of the
    learned run's root launch."""
    import numpy as np
    import torch

    import paper_1707_05594_amd as tk
    import paper_1707_05594_amd.costmodel as cm
    import synth
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    T, info = synth.workload("planted_64x48x40x32x24x16_f32")
    L, K = info["L"], info["K"]
    Td = torch.from_numpy(T).to(dev)
    del T
    torch.cuda.synchronize()
    log(f"six-mode: generated in {time.perf_counter() - t0:.1f}s")

    def run(plan):
        ctx = tk.hooi_init(Td, K, plan=plan, compute="fp32")
        F0 = ctx.factors()
        ctx.iterate(max(1, warmup))
        ctx.set_factors(F0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        errs = ctx.iterate(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / steps
        node = [sorted(x) for x in zip(*[ctx.profile_tree() for _ in range(3)])]
        med = [v[1] for v in node]
        return ctx, dt, errs, med

    plain = tk.ttm_tree_plan(L, K)
    ctx, dt_p, errs_p, med_p = run(plain)
    e_p = ctx.error_explicit()
    del ctx
    # cost model: node and root-pair timings of random shapes, trained on the GPU
    t2 = time.perf_counter()
    X, y, rows, prow = cm.training_set(n_shapes=10, n_pairs=48, seed=1)
    model, losses = cm.train(X, y, steps=3000, lr=3e-3)
    plan = tk.ttm_tree_plan(L, K, "dp", topk=8)
    chosen, pred = plan.learned(model, "f32", "fp32", margin=0.02)
    tiles = plan.tiles(chosen)
    t_model = time.perf_counter() - t2
    ctx, dt_l, errs_l, med_l = run(plan)
    e_l = ctx.error_explicit()
    nodes = plan.nodes(chosen)
    roots = [i for i, n in enumerate(nodes) if n["parent"] < 0 and not n["is_leaf"]]
    fused = tk.TK_TILE_PAIR in tiles
    root_ms = sum(med_l[i] for i in roots)
    card_T = 1
    for x in L:
        card_T *= x
    root_bytes = (4 * card_T * (1 if fused else len(roots)) +
                  sum(4 * nodes[i]["out_card"] + 4 * L[nodes[i]["mode"]] * K[nodes[i]["mode"]]
                      for i in roots))
    ach = root_bytes / (root_ms * 1e-3) / 1e9
    res = {"workload": "planted 64x48x40x32x24x16 FP32, ranks 8,8,6,6,4,4, core 1/(i1+..+i6), "
                       "1e-3 rel noise, HOSVD start",
           "plain_dp": {"tree": plain.string(), "tree_macs": plain.cost(),
                        "value": round(1.0 / dt_p, 3), "unit": "HOOI iters/s",
                        "ms_per_step": round(1e3 * dt_p, 4), "tree_ms_per_pass": round(sum(med_p), 4),
                        "rel_err": errs_p[-1], "rel_err_explicit": e_p,
                        "iteration_roofline": iteration_roofline(plain, 1e3 * dt_p)},
           "learned": {"chosen_rank": chosen, "tree": plan.string(chosen),
                       "tree_macs": plan.cost(chosen), "fused_root_pair": fused,
                       "predicted_tree_ms": round(float(pred[chosen]), 4),
                       "value": round(1.0 / dt_l, 3), "unit": "HOOI iters/s",
                       "ms_per_step": round(1e3 * dt_l, 4), "tree_ms_per_pass": round(sum(med_l), 4),
                       "rel_err": errs_l[-1], "rel_err_explicit": e_l,
                       "speedup_vs_plain_dp": round(dt_p / dt_l, 3),
                       "model": {"node_rows": len(rows), "pair_rows": len(prow),
                                 "final_loss": float(losses[-1]),
                                 "harvest_and_train_s": round(t_model, 1)},
                       "iteration_roofline": iteration_roofline(plan, 1e3 * dt_l)},
           "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": ("ttm_pair_tail_f32 (both root children, T read once)" if fused
                                   else "root TTMs"),
                        "avg_ms": round(root_ms, 4), "bytes_per_launch": int(root_bytes)}}
    log(f"six-mode: plain DP {1.0 / dt_p:.1f} it/s ({1e3 * dt_p:.3f} ms), learned "
        f"{1.0 / dt_l:.1f} it/s ({1e3 * dt_l:.3f} ms, rank {chosen}, fused {fused}); errors "
        f"{e_p:.9e} / {e_l:.9e}")
    del ctx, Td
    torch.cuda.empty_cache()
    return res


def real_shapes_leg(steps=2):
    """The paper's real-tensor shapes (Sec. 6.1 table: HCCI, TJLR, SP) filled
    with uniform random data, FP32, DP tree, HOSVD start: per shape the HOOI
    invocation time, the tree pass alone and its TTM rate against the FP32
    MFMA peak (ranks up to 306: the contractions are compute-heavy here), and
    the rest of the invocation (Grams, gap-free eigensolves, core)."""
    import torch

    import paper_1707_05594_amd as tk
    import synth
    dev = torch.device("cuda:0")
    out = {}
    for name, (L, K) in synth.REAL_TENSORS.items():
        t0 = time.perf_counter()
        Td = synth.real_tensor_device(name, dev)
        plan = tk.ttm_tree_plan(L, K)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx = tk.hooi_init(Td, K, plan=plan, compute="fp32")
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t1
        ctx.iterate(1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        errs = ctx.iterate(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t2) / steps
        node = [sorted(x)[1] for x in zip(*[ctx.profile_tree() for _ in range(3)])]
        nodes = plan.nodes()
        tree_ms = sum(node)
        ttm_ms = sum(t for t, nd in zip(node, nodes) if not nd["is_leaf"])
        flops = 2.0 * plan.cost()
        tf = flops / (ttm_ms * 1e-3) / 1e12
        card = 1
        for x in L:
            card *= x
        out[name] = {"L": list(L), "K": list(K), "elements": card, "tree": plan.string(),
                     "tree_macs": plan.cost(), "hosvd_s": round(t_init, 3),
                     "value": round(1.0 / dt, 4), "unit": "HOOI iters/s",
                     "ms_per_step": round(1e3 * dt, 2), "tree_ms_per_pass": round(tree_ms, 2),
                     "ttm_ms_per_pass": round(ttm_ms, 2), "ttm_tflops": round(tf, 2),
                     "ttm_frac_fp32_mfma_peak": round(tf / FP32_MFMA_PEAK_TFLOPS, 4),
                     "rest_ms_per_step": round(1e3 * dt - tree_ms, 2),
                     "rel_err": errs[-1]}
        log(f"{name}: {1e3 * dt:.1f} ms per invocation (tree {tree_ms:.1f} ms, TTMs {ttm_ms:.1f} "
            f"ms at {tf:.1f} TFLOP/s = {tf / FP32_MFMA_PEAK_TFLOPS:.3f} of FP32 MFMA peak), "
            f"HOSVD {t_init:.2f} s, total leg {time.perf_counter() - t0:.1f} s")
        del ctx, Td
        torch.cuda.empty_cache()
    return out


def sthosvd_leg(Td, K, plan, steps):
    """HOSVD against STHOSVD starts on the benchmark tensor: start time, the
    FP64 explicit residual of each start and after `steps` invocations."""
    import torch

    import paper_1707_05594_amd as tk
    res = {}
    for init in ("hosvd", "sthosvd"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = tk.hooi_init(Td, K, plan=plan, compute="fp32", init=init)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        e0 = ctx.error_explicit()
        ctx.iterate(steps)
        e1 = ctx.error_explicit()
        res[init] = {"init_ms": round(1e3 * dt, 2), "rel_err_start": e0,
                     "rel_err_after_%d" % steps: e1}
        log(f"{init}: start {1e3 * dt:.1f} ms, error {e0:.9e} -> {e1:.9e} after {steps}")
        del ctx
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--skip-mixed", action="store_true")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--skip-five-mode", action="store_true")
    ap.add_argument("--skip-sthosvd", action="store_true")
    ap.add_argument("--skip-six-mode", action="store_true")
    ap.add_argument("--skip-real-shapes", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="finish with three device-to-device copies of BYTES bytes "
                         "(dispatches of known size that calibrate the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1707_05594_amd as tk
    import synth

    t0 = time.perf_counter()
    T, info = synth.workload(WORKLOAD)
    L, K = info["L"], info["K"]
    log(f"generated {WORKLOAD} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    Td = torch.from_numpy(T).to(dev)
    torch.cuda.synchronize()
    plan = tk.ttm_tree_plan(L, K)
    ctx = tk.hooi_init(Td, K, plan=plan, compute="fp32")
    F0 = ctx.factors()
    log(f"plan {plan.string()} macs {plan.cost()}")

    if args.warmup > 0:
        ctx.iterate(args.warmup)
    ctx.set_factors(F0)  # timed run starts from the HOSVD factors again
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    errs = ctx.iterate(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ms_per_step = 1e3 * elapsed / args.steps
    its = args.steps / elapsed
    log(f"{args.steps} steps in {elapsed * 1e3:.2f} ms, errors {errs}")
    log(f"eigensolver steps per mode (last update): {ctx.eig_iterations()}")

    roof, node_ms = root_ttm_roofline(ctx, plan)
    tree_ms = sum(node_ms)
    tree_macs = plan.cost()
    gflops_step = 2.0 * tree_macs / (ms_per_step * 1e-3) / 1e9
    gflops_tree = 2.0 * tree_macs / (tree_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(its, 3),
        "unit": "HOOI iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "planted 200x200x200x200 FP32, Tucker rank 20/mode, 1e-3 rel "
                               "noise, HOSVD start, DP-optimal TTM-tree",
                   "L": list(L), "K": list(K), "tree": plan.string(), "tree_macs": tree_macs},
        "ttm_gflops": round(gflops_step, 1),
        "ttm_gflops_tree_only": round(gflops_tree, 1),
        "ttm_frac_fp32_mfma_peak": round(gflops_step / (FP32_MFMA_PEAK_TFLOPS * 1e3), 4),
        "rel_err": errs[-1],
        "roofline": roof,
        "iteration_roofline": iteration_roofline(plan, ms_per_step),
    }

    if not args.skip_mixed:
        # same tensor stored as BF16; factors from each reduced-precision run are
        # scored against the FP32 tensor with the FP64 explicit residual
        e32 = ctx.error_explicit()
        out["rel_err_explicit"] = e32
        Tb = Td.to(torch.bfloat16)
        mixed = []
        for compute in ("bf16x3", "bf16"):
            ctxb = tk.hooi_init(Tb, K, plan=plan, compute=compute, F0=F0)
            ctxb.iterate(max(1, args.warmup))
            ctxb.set_factors(F0)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            errs_b = ctxb.iterate(args.steps)
            torch.cuda.synchronize()
            eb = time.perf_counter() - t2
            ctx.set_factors(ctxb.factors())
            err_vs_f32 = ctx.error_explicit()
            mixed.append({"storage": "bf16 T", "compute": f"{compute} MFMA (core at FP32), "
                                                            "FP64 eigensolver",
                          "value": round(args.steps / eb, 3), "unit": "HOOI iters/s",
                          "ms_per_step": round(1e3 * eb / args.steps, 4),
                          "speedup_vs_fp32": round((args.steps / eb) / its, 3),
                          "rel_err_vs_fp32_T": err_vs_f32, "rel_err_fp32_run": e32,
                          "rel_err_vs_bf16_T": errs_b[-1]})
            log(f"bf16 storage, {compute}: {mixed[-1]['value']} it/s, error vs FP32 T "
                f"{err_vs_f32:.6e} (FP32 run {e32:.6e})")
            del ctxb
        out["mixed"] = mixed
        del Tb

    if not args.skip_sthosvd:
        out["sthosvd_vs_hosvd"] = sthosvd_leg(Td, K, plan, 3)

    if not args.skip_five_mode:
        out["bf16_storage_80x80x80x80x80"] = five_mode_bf16_leg(args.steps, args.warmup)

    if not args.skip_six_mode:
        out["six_mode_64x48x40x32x24x16"] = six_mode_leg(args.steps, args.warmup)
    if not args.skip_real_shapes:
        out["real_shapes"] = real_shapes_leg()

    if not args.skip_batch:
        out["batch"] = batch_leg(args.steps, args.warmup)

    if not args.skip_cpu_baseline:
        log("timing the FP64 oracle on one HOOI invocation ...")
        out["cpu_baseline"] = cpu_baseline(T, K, F0)
    if args.copy_calibration > 0:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 4 * n
        del src, dst
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
