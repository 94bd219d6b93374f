"""Batched HOOI on the GPU (grouped persistent TTM levels, grouped Grams,
batched eigensolves, HIP-graph replay) against the FP64 oracle per tensor,
against the single-tensor engine, and graph replays against eager runs.

Bars: FP32 TTMs with relative noise 1e-2, so the identity error is good to
~1e-4 relative (FP32 ||G||^2 moves e^2 by ~1e-8): 1e-3; factor subspaces
within 1e-4 of the oracle's (FP32 leaves, eigen-gap of the planted ranks);
graph replays and eager runs, and every persistent grid size, give bitwise
identical factors (each work item is computed the same way wherever it runs)."""
import numpy as np
import pytest

import synth
from oracle import hooi as O
from tests.gpu_util import subspace_dist, torch_dev

pytestmark = pytest.mark.gpu
tk = pytest.importorskip("paper_1707_05594_amd")


def _batch(count, dtype="f32", seed=0, lmin=8, lmax=40, kmin=2, kmax=6, noise=1e-2):
    torch, dev = torch_dev()
    shapes = synth.batch_shapes(count, cfg=5, seed_idx=seed, lmin=lmin, lmax=lmax, kmin=kmin,
                                kmax=kmax)
    host, devs = [], []
    for i, (L, K) in enumerate(shapes):
        T, _ = synth.planted(L, K, noise=noise, noise_kind="rel", dtype=dtype, cfg=5, idx=i)
        host.append(T)
        if dtype == "bf16":
            devs.append(torch.from_numpy(T.view(np.int16)).view(torch.bfloat16).to(dev))
        else:
            devs.append(torch.from_numpy(T).to(dev))
    torch.cuda.synchronize()
    return shapes, host, devs


def test_batch_matches_oracle_per_tensor():
    shapes, host, devs = _batch(12, seed=1)
    print(f"batch of {len(shapes)}: {shapes[:3]} ...", flush=True)
    b = tk.Batch(devs, [K for _, K in shapes])
    print(f"stats {b.stats()}", flush=True)
    for i, (L, K) in enumerate(shapes):
        F0 = O.hosvd(host[i].astype(np.float64), K)
        for n in range(len(L)):
            assert subspace_dist(b.factor(i, n), F0[n]) < 1e-8, (i, n)
    iters = 3
    errs = b.iterate(iters)
    cur = b.error()
    for i, (L, K) in enumerate(shapes):
        T64 = host[i].astype(np.float64)
        Fo, Go, eo = O.hooi(T64, K, iters)
        e_hosvd = O.rel_error_explicit(T64, O.new_core(T64, O.hosvd(T64, K)), O.hosvd(T64, K))
        assert abs(errs[0, i] - e_hosvd) < 1e-3 * e_hosvd
        for t in range(1, iters):
            assert abs(errs[t, i] - eo[t - 1]) < 1e-3 * eo[t - 1], (i, t)
        assert abs(cur[i] - eo[-1]) < 1e-3 * eo[-1]
        for n in range(len(L)):
            assert subspace_dist(b.factor(i, n), Fo[n]) < 1e-4, (i, n)


def _real_shape_sample(count, dtype):
    """A seeded sample of the 512-tensor batch itself (3- and 4-mode tensors,
    L_n uniform in [32, 128], K_n uniform in [4, 16], 1e-3 relative noise):
    its largest tensor plus count - 1 others, each generated with the seed it
    has in the whole batch."""
    torch, dev = torch_dev()
    shapes = synth.batch_shapes(512, cfg=5)
    sizes = [int(np.prod(L)) for L, _ in shapes]
    big = int(np.argmax(sizes))
    g = np.random.default_rng(512)
    rest = [i for i in range(len(shapes)) if i != big]
    pick = [big] + sorted(int(i) for i in g.choice(rest, count - 1, replace=False))
    sub = [shapes[i] for i in pick]
    # the sample covers what the small-shape tests do not: modes above 64
    # (subspace eigensolves, several 64-row Gram tiles), ranks above 12,
    # three- and four-mode tensors
    assert max(max(L) for L, _ in sub) > 120 and max(max(K) for _, K in sub) >= 14
    assert {len(L) for L, _ in sub} == {3, 4}
    host, devs = [], []
    for i in pick:
        L, K = shapes[i]
        T, _ = synth.planted(L, K, noise=1e-3, noise_kind="rel", dtype=dtype, cfg=5, idx=i)
        host.append(T)
        if dtype == "bf16":
            devs.append(torch.from_numpy(T.view(np.int16)).view(torch.bfloat16).to(dev))
        else:
            devs.append(torch.from_numpy(T).to(dev))
    torch.cuda.synchronize()
    return pick, sub, host, devs


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batch_real_shapes_match_oracle(dtype):
    """Sixteen tensors of the 512-tensor batch, its largest included, through
    the batched engine against the FP64 oracle (on the exact upcast of the
    stored values), three invocations from HOSVD.

    Bars: HOSVD subspaces 1e-8; after three invocations subspaces 1e-4 (FP32
    leaves, planted gap); the oracle's FP64 explicit residual of the GPU's
    factors (with their optimal core) within 1e-6 relative of the oracle's
    own error (the error is stationary in the factors).  The engine's
    per-invocation errors come from the identity e^2 = 1 - ||G||^2 / ||T||^2
    with an FP32 core of |G| entries; the rounding of the chain that forms it
    (about u sqrt(sum L) per entry, u = 2^-24, independent between entries)
    moves ||G||^2 / ||T||^2 by about 2 u sqrt(sum L) / sqrt(|G|), i.e. e by
    u sqrt(sum L) / (sqrt(|G|) e^2) relative: 9% for an 80-entry core at
    e = 1e-3, under 1% for the larger ones.  They are checked within four
    times that figure (the explicit residual is the precise value)."""
    pick, shapes, host, devs = _real_shape_sample(16, dtype)
    print(f"{dtype} sample {pick}: {shapes}", flush=True)
    b = tk.Batch(devs, [K for _, K in shapes])
    iters = 3
    F_h = [[b.factor(i, n) for n in range(len(L))] for i, (L, _) in enumerate(shapes)]
    errs = b.iterate(iters)
    cur = b.error()
    for i, (L, K) in enumerate(shapes):
        T64 = O.as_f64(host[i], dtype)
        F0 = O.hosvd(T64, K)
        for n in range(len(L)):
            assert subspace_dist(F_h[i][n], F0[n]) < 1e-8, (pick[i], n)
        Fo, Go, eo = O.hooi(T64, K, iters, F0=F0)
        Fg = [b.factor(i, n) for n in range(len(L))]
        e_g = O.rel_error_explicit(T64, O.new_core(T64, Fg), Fg)
        dist = max(subspace_dist(Fg[n], Fo[n]) for n in range(len(L)))
        print(f"tensor {pick[i]} L={L} K={K}: oracle error {eo[-1]:.9e}, GPU factors "
              f"{e_g:.9e}, engine {cur[i]:.9e}, subspace distance {dist:.2e}", flush=True)
        assert dist < 1e-4, pick[i]
        assert abs(e_g - eo[-1]) < 1e-6 * eo[-1], pick[i]
        noise = 2.0 ** -24 * np.sqrt(sum(L)) / (np.sqrt(np.prod(K)) * eo[-1] ** 2)
        for t in range(1, iters):
            assert abs(errs[t, i] - eo[t - 1]) < 4 * noise * eo[t - 1], (pick[i], t, noise)
        assert abs(cur[i] - eo[-1]) < 4 * noise * eo[-1], (pick[i], noise)


def test_batch_matches_single_tensor_engine():
    shapes, host, devs = _batch(6, seed=2)
    b = tk.Batch(devs, [K for _, K in shapes])
    b.iterate(2)
    for i, (L, K) in enumerate(shapes):
        ctx = tk.hooi_init(devs[i], K, compute="fp32")
        ctx.iterate(2)
        for n in range(len(L)):
            assert subspace_dist(b.factor(i, n), ctx.factor(n)) < 1e-5, (i, n)


def test_graph_replays_equal_eager_runs_and_tuning_keeps_results():
    shapes, host, devs = _batch(10, seed=3)
    K = [k for _, k in shapes]
    eager = tk.Batch(devs, K)
    eager.use_graph(False)
    graph = tk.Batch(devs, K)
    tuned = tk.Batch(devs, K)
    bpc, ms = tuned.tune()
    print(f"tuned blocks/CU {bpc}, pass times {ms[:4]}, other row body {ms[4]}", flush=True)
    assert bpc in (1, 2, 3, 4)
    # the two row bodies accumulate the same MFMAs in the same order, so either
    # choice reproduces the eager run bitwise (checked below)
    e_eager = eager.iterate(4)
    # graph replays one at a time, with eager work (error evaluations) between them
    parts = []
    for _ in range(4):
        parts.append(graph.iterate(1))
        graph.error()
    e_graph = np.concatenate(parts)
    e_tuned = tuned.iterate(4)
    np.testing.assert_array_equal(graph.factors(), eager.factors())
    np.testing.assert_array_equal(tuned.factors(), eager.factors())
    np.testing.assert_array_equal(e_graph, e_eager)
    np.testing.assert_array_equal(e_tuned, e_eager)


def test_batch_bf16_storage():
    shapes, host, devs = _batch(6, dtype="bf16", seed=4)
    b = tk.Batch(devs, [K for _, K in shapes])
    b.iterate(2)
    cur = b.error()
    for i, (L, K) in enumerate(shapes):
        T64 = O.as_f64(host[i], "bf16")
        Fo, Go, eo = O.hooi(T64, K, 2)
        assert abs(cur[i] - eo[-1]) < 1e-3 * eo[-1]
        for n in range(len(L)):
            assert subspace_dist(b.factor(i, n), Fo[n]) < 1e-4


def test_batch_rejects_bad_input():
    torch, dev = torch_dev()
    T = torch.zeros((8, 8, 8), dtype=torch.float32, device=dev)
    with pytest.raises(tk.TuckerError) as e:
        tk.Batch([T], [(2, 2, 20)])
    assert e.value.code == tk.TK_EINVAL
    with pytest.raises(tk.TuckerError) as e:
        tk.Batch([torch.zeros((40, 40, 40), dtype=torch.float32, device=dev)], [(20, 20, 20)])
    assert e.value.code == tk.TK_EUNSUPPORTED


def test_resume_from_factors_matches_to_rounding():
    """Full solves (L <= 64) keep their eigenbasis from one invocation to the
    next as a warm start; setting the factors restarts those bases from the
    identity.  Any orthonormal start gives the same eigenvectors up to
    rounding, so a batch resumed from saved factors follows the uninterrupted
    run to rounding (the FP32 copies of the factors, hence every leaf, stay
    equal)."""
    shapes, host, devs = _batch(8, seed=4)
    K = [k for _, k in shapes]
    a = tk.Batch(devs, K)
    a.iterate(2)
    F = a.factors()
    a.iterate(2)
    b = tk.Batch(devs, K)
    b.set_factors(F)
    b.iterate(2)
    for i, (L, _) in enumerate(shapes):
        for n in range(len(L)):
            assert subspace_dist(a.factor(i, n), b.factor(i, n)) < 1e-9, (i, n)
    np.testing.assert_allclose(a.error(), b.error(), rtol=1e-9)
