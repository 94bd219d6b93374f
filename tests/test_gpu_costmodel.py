"""Learned tree selection on the GPU: the MLP's forward, gradient and Adam
steps against the float64 oracle (oracle.mlp), and the selection itself on the
six-mode 64x48x40x32x24x16 tensor (ranks 8,8,6,6,4,4).

Bars: forward and loss within 1e-5 relative (FP32 sums of at most 32 terms);
gradients within 1e-4 normwise (FP32 accumulation over the batch); five Adam
steps within 1e-3 normwise of the oracle's parameter change.  The selection
must not be slower than the DP optimum with automatic kernels by more than
the timing noise (3%)."""
import numpy as np
import pytest

import synth
from oracle import mlp as M
from tests.gpu_util import rel_err, torch_dev

pytestmark = pytest.mark.gpu
tk = pytest.importorskip("paper_1707_05594_amd")
cm = pytest.importorskip("paper_1707_05594_amd.costmodel")

D, H = 12, 32


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
    # training data: node shapes of the 8 best trees of random tensors (not this one)
    views = []
    for Ls, Ks in cm.random_shapes(10, seed=1):
        views += cm.candidate_views(Ls, Ks, topk=8)
    print(f"timing {len(views)} node shapes x 3 kernels", flush=True)
    X, y, _ = cm.measure(views)
    model, losses = cm.train(X, y, steps=3000, lr=3e-3)
    print(f"training loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.25 * losses[0]
    # held-out check: this tensor's candidate nodes
    Xc, yc, _ = cm.measure(cm.candidate_views(L, K, topk=8))
    pred = model.forward(Xc)
    corr = float(np.corrcoef(pred, yc)[0, 1])
    print(f"held-out correlation of log times {corr:.3f}", flush=True)
    assert corr > 0.9
    plan = tk.ttm_tree_plan(L, K, "dp", topk=8)
    chosen, pred_ms = plan.learned(model, "f32", "fp32", margin=0.02)
    print(f"chosen rank {chosen} tiles {plan.tiles(chosen)} predicted {pred_ms}", flush=True)
    T, _ = synth.workload("planted_64x48x40x32x24x16_f32")
    Td = torch.from_numpy(T).to(dev)

    def tree_ms(rank, tiles=None):
        p = tk.ttm_tree_plan(L, K, "dp", topk=8)
        p.select(rank)
        if tiles is not None:
            p.set_tiles(rank, tiles)
        ctx = tk.hooi_init(Td, K, plan=p, compute="fp32")
        ms = [sum(ctx.profile_tree()) for _ in range(5)]
        return float(np.median(ms))

    t_dp = tree_ms(0)
    t_learned = tree_ms(chosen, plan.tiles(chosen))
    print(f"tree time: DP optimum {t_dp:.3f} ms, learned choice {t_learned:.3f} ms", flush=True)
    assert t_learned <= 1.03 * t_dp
