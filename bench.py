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


def recorded_traffic():
    """HBM bytes per root-TTM launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel
    sources have changed since the counters were taken."""
    import hashlib
    try:
        text = open(COUNTERS).read().splitlines()
    except OSError:
        return None
    traffic, digest, files = None, None, []
    for line in text:
        line = line.strip()
        if line.startswith("traffic_bytes_per_launch:"):
            traffic = int(line.split(":")[1])
        elif line.startswith("kernel_source_sha256_16:"):
            parts = line.split(":", 1)[1].split()
            digest = parts[0]
            files = [f.strip("()") for f in parts[1:]]
    if traffic is None or digest is None or not files:
        return None
    h = hashlib.sha256()
    for f in files:
        try:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        except OSError:
            return None
    return traffic if h.hexdigest()[:16] == digest else None


def root_ttm_roofline(ctx, plan, reps=3):
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
        per_launch.append(4 * (n["in_card"] + n["out_card"]) + 4 * L[n["mode"]] * K[n["mode"]])
    bytes_per_launch = sum(per_launch) / len(per_launch)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=recorded_traffic(),
                kernel="ttm_wide_f32 (root nodes, reads T)", launches=len(times),
                avg_ms=round(avg_ms, 4), bytes_per_launch=int(bytes_per_launch)), ms


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
                        "rel_err_explicit": ctx.error_explicit()}
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
    ctxs = [tk.hooi_init(devs[i], ranks[i], compute="fp32") for i in sub]
    for c in ctxs:
        c.iterate(1)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for c in ctxs:
        c.iterate(steps)
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t3) / steps
    res = {"workload": "512 planted tensors, 3- or 4-mode, L in [32,128], K in [4,16], 1e-3 rel "
                       "noise, FP32, HOSVD start, DP tree each",
           "elements": int(elems), "value": round(1.0 / dt, 3), "unit": "batch HOOI iters/s",
           "ms_per_step": round(1e3 * dt, 4), "tree_macs": st["tree_macs"],
           "tree_bytes": st["tree_bytes"], "levels": st["levels"], "ttm_items": st["ttm_items"],
           "tree_GBps_at_step_time": round(st["tree_bytes"] / dt / 1e9, 1),
           "frac_hbm_peak": round(st["tree_bytes"] / dt / 1e9 / HBM_PEAK_GBS, 4),
           "tuned_blocks_per_cu": bpc, "tune_level_ms": [round(float(x), 4) for x in tune_ms],
           "rel_err_median": float(np.median(cur)), "rel_err_max": float(np.max(cur)),
           "first_%d" % seq_count: {"batched_ms_per_step": round(1e3 * dt_b, 4),
                                    "one_context_each_ms_per_step": round(1e3 * dt_s, 4),
                                    "speedup": round(dt_s / dt_b, 2)}}
    log(f"batch: {res['value']} it/s ({res['ms_per_step']} ms), tree {st['tree_bytes']/1e9:.1f} GB "
        f"-> {res['tree_GBps_at_step_time']} GB/s; first {seq_count}: batched {1e3*dt_b:.2f} ms vs "
        f"one context each {1e3*dt_s:.2f} ms")
    del b, bs, ctxs, devs
    torch.cuda.empty_cache()
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

    if not args.skip_five_mode:
        out["bf16_storage_80x80x80x80x80"] = five_mode_bf16_leg(args.steps, args.warmup)

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
