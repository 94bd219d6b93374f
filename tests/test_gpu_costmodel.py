"""Learned tree selection on the GPU: the MLP's forward, gradient and Adam
steps against the float64 oracle (oracle.mlp), and the selection itself on the
six-mode 64x48x40x32x24x16 tensor (ranks 8,8,6,6,4,4).

Bars: forward and loss within 1e-5 relative (FP32 sums of at most 32 terms);
gradients within 1e-4 normwise (FP32 accumulation over the batch); five Adam
steps within 1e-3 normwise of the oracle's parameter change.  On the six-mode
tensor the candidates include running the DP tree's two root children (the
trailing modes) as one pass over T; the test measures the plain DP tree
(separate root TTMs, automatic kernels) against the learned choice and asserts
the learned choice at least 10% faster per HOOI invocation, at the same
explicit error (1e-6 relative: the same decomposition up to FP32 rounding)."""
import time

import numpy as np
import pytest

import synth
from oracle import mlp as M
from tests.gpu_util import rel_err, torch_dev

pytestmark = pytest.mark.gpu
tk = pytest.importorskip("paper_1707_05594_amd")
cm = pytest.importorskip("paper_1707_05594_amd.costmodel")

D, H = 13, 32


def _data(n, seed):
    g = np.random.default_rng(seed)
    X = (g.standard_normal((n, D)) * 2 + 3).astype(np.float32)
    y = (np.sin(X[:, 0]) + 0.1 * X[:, 1] * X[:, 2]).astype(np.float32)
    return X, y


def _model(X, seed=0):
    p = cm.init_params(D, H, seed)
    m = tk.MLP(D, H, p)
    mu = X.mean(axis=0).astype(np.float32)
    sg = X.std(axis=0).astype(np.float32)
    m.set_norm(mu, sg)
    return m, p.astype(np.float64), mu.astype(np.float64), sg.astype(np.float64)


def test_mlp_forward_and_gradient_match_oracle():
    torch_dev()
    X, y = _data(300, 1)
    m, p, mu, sg = _model(X)
    got = m.forward(X)
    want, _ = M.forward(p, X, mu, sg, D, H)
    assert rel_err(got, want) < 1e-5
    loss, g = m.loss_grad(X, y)
    loss_o, g_o = M.loss_grad(p, X, y, mu, sg, D, H)
    assert abs(loss - loss_o) < 1e-5 * loss_o
    assert rel_err(g, g_o) < 1e-4


def test_mlp_fit_norm_standardises_like_the_definition():
    """tk_mlp_fit_norm: the oracle's forward with the per-feature mean and
    population deviation of X (a constant feature keeps sigma = 1)."""
    torch_dev()
    X, _ = _data(300, 4)
    X[:, 5] = 7.0  # constant feature
    p = cm.init_params(D, H, 5)
    m = tk.MLP(D, H, p)
    m.fit_norm(X)
    X64 = X.astype(np.float64)
    mu = X64.mean(axis=0)
    sg = X64.std(axis=0)
    sg[5] = 1.0
    # the library rounds mu and sigma to FP32 as set_norm stores them
    want, _ = M.forward(p.astype(np.float64), X, mu.astype(np.float32).astype(np.float64),
                        sg.astype(np.float32).astype(np.float64), D, H)
    assert rel_err(m.forward(X), want) < 1e-5
    with pytest.raises(tk.TuckerError):
        m.fit_norm(X[:0])


def test_mlp_adam_steps_match_oracle():
    torch_dev()
    X, y = _data(257, 2)
    m, p0, mu, sg = _model(X, seed=3)
    losses = m.train(X, y, 5, 1e-2)
    p, mo, vo = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    losses_o = []
    for t in range(1, 6):
        l, g = M.loss_grad(p, X, y, mu, sg, D, H)
        losses_o.append(l)
        p, mo, vo = M.adam(p, g, mo, vo, t, 1e-2)
    np.testing.assert_allclose(losses, losses_o, rtol=1e-4)
    assert rel_err(m.params() - p0, p - p0) < 1e-3


def test_learned_selection_on_six_mode_tensor():
    torch, dev = torch_dev()
    L, K = (64, 48, 40, 32, 24, 16), (8, 8, 6, 6, 4, 4)
    # training data: node shapes of the 8 best trees of random tensors (not this
    # one), the root pairs a pair kernel takes, and random trailing-pair views
    X, y, rows, prow = cm.training_set(n_shapes=10, n_pairs=48, seed=1)
    print(f"timed {len(rows)} node rows and {len(prow)} fused root pairs", flush=True)
    assert len(prow) >= 8
    model, losses = cm.train(X, y, steps=3000, lr=3e-3)
    print(f"training loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.25 * losses[0]
    # held-out check: this tensor's candidate nodes
    Xc, yc, _ = cm.measure(cm.candidate_views(L, K, topk=8))
    pred = model.forward(Xc)
    corr = float(np.corrcoef(pred, yc)[0, 1])
    print(f"held-out correlation of log times {corr:.3f}", flush=True)
    assert corr > 0.9
    # the model's view of the DP tree's root level: separate TTMs or one pass
    pv = cm.root_pair_view(L, K, tk.ttm_tree_plan(L, K), 0)
    A, Lp, M, Lq, B, Kp, Kq = pv
    sep = [tk.ttm_features(A, Lp, M * Lq * B, Kp, "f32", "fp32", t) for t in range(tk.TK_TILE_COUNT)]
    sep_q = [tk.ttm_features(A * Lp * M, Lq, B, Kq, "f32", "fp32", t)
             for t in range(tk.TK_TILE_COUNT)]
    p_sep = (np.exp(model.forward(np.array(sep, np.float32))).min() +
             np.exp(model.forward(np.array(sep_q, np.float32))).min())
    p_pair = float(np.exp(model.forward(np.array([tk.pair_features(*pv)], np.float32)))[0])
    print(f"root level predicted: separate {p_sep:.3f} ms, one pass {p_pair:.3f} ms", flush=True)
    plan = tk.ttm_tree_plan(L, K, "dp", topk=8)
    chosen, pred_ms = plan.learned(model, "f32", "fp32", margin=0.02)
    print(f"chosen rank {chosen} tiles {plan.tiles(chosen)} predicted {pred_ms}", flush=True)
    T, _ = synth.workload("planted_64x48x40x32x24x16_f32")
    Td = torch.from_numpy(T).to(dev)

    def run(rank, tiles=None):
        """Median tree-pass time (node sum) and HOOI time per invocation (the
        eigensolves overlap the pass on a side stream), plus the explicit
        error after the timed invocations."""
        p = tk.ttm_tree_plan(L, K, "dp", topk=8)
        p.select(rank)
        if tiles is not None:
            p.set_tiles(rank, tiles)
        ctx = tk.hooi_init(Td, K, plan=p, compute="fp32")
        tree = float(np.median([sum(ctx.profile_tree()) for _ in range(5)]))
        ctx.iterate(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.iterate(20)
        torch.cuda.synchronize()
        it = (time.perf_counter() - t0) / 20 * 1e3
        return tree, it, ctx.error_explicit()

    tree_dp, it_dp, e_dp = run(0)
    tree_l, it_l, e_l = run(chosen, plan.tiles(chosen))
    print(f"DP optimum: tree {tree_dp:.3f} ms, HOOI {it_dp:.3f} ms/invocation, error {e_dp:.9e}",
          flush=True)
    print(f"learned (rank {chosen}): tree {tree_l:.3f} ms, HOOI {it_l:.3f} ms/invocation, "
          f"error {e_l:.9e}; gain {it_dp / it_l:.3f}x", flush=True)
    assert tk.TK_TILE_PAIR in plan.tiles(chosen)
    assert it_l <= 0.9 * it_dp
    assert abs(e_l - e_dp) <= 1e-6 * e_dp
