"""End-to-end HOOI on the GPU through the C ABI against the FP64 oracle.

Bars (from the arithmetic): leaves element-wise within the first-order bound
of their chain of TTMs relative to the chain over |T| and |F| (tests/gpu_util.py
states the per-precision bounds); FP64 errors within 1e-10 relative; factors
compared basis-free (projector distance) and, where the planted eigen-gap makes
them unique, element-wise after the sign rule."""
import numpy as np
import pytest

import synth
from oracle import hooi as O
from tests.gpu_util import (abs_chain, assert_elementwise, chain_tol, rel_err, subspace_dist,
                            to_dev, torch_dev)

pytestmark = pytest.mark.gpu
tk = pytest.importorskip("paper_1707_05594_amd")


def _device_T(T_stored, dtype):
    torch, dev = torch_dev()
    if dtype == "bf16":
        return torch.from_numpy(np.ascontiguousarray(T_stored).view(np.int16)).view(
            torch.bfloat16).to(dev)
    return torch.from_numpy(np.ascontiguousarray(T_stored)).to(dev)


def test_64cube_fp64_hosvd_and_iterations_match_oracle():
    T, info = synth.workload("planted_64x64x64_r8_f64")
    K = info["K"]
    print("64^3 fp64 HOSVD + 10 iterations", flush=True)
    Td = _device_T(T, "f64")
    ctx = tk.hooi_init(Td, K, compute="fp64")
    F0 = O.hosvd(T, K)
    for n in range(3):
        Fg = ctx.factor(n)
        assert subspace_dist(Fg, F0[n]) < 1e-10
        assert np.abs(Fg - F0[n]).max() < 1e-9
    errs = ctx.iterate(10)
    Fo, Go, errs_o = O.hooi(T, K, 10)
    np.testing.assert_allclose(errs, errs_o, rtol=1e-10)
    for n in range(3):
        assert subspace_dist(ctx.factor(n), Fo[n]) < 1e-10
    assert rel_err(ctx.core(), Go) < 1e-9
    e_id, nT, nG = ctx.error()
    assert abs(e_id - errs[-1]) < 1e-15
    assert abs(ctx.error_explicit() - errs_o[-1]) < 1e-10 * errs_o[-1]
    # monotone on this planted tensor (Jacobi form; flat to roundoff)
    for a, b in zip(errs, errs[1:]):
        assert b <= a + 1e-12


def test_naive_chain_and_dp_tree_agree():
    T, info = synth.workload("planted_64x64x64_r8_f64")
    K = info["K"]
    Td = _device_T(T, "f64")
    e_dp = tk.hooi_init(Td, K, compute="fp64").iterate(3)
    e_ch = tk.hooi_init(Td, K, compute="fp64", plan=tk.ttm_tree_plan(T.shape, K, "chain")).iterate(3)
    e_bal = tk.hooi_init(Td, K, compute="fp64",
                         plan=tk.ttm_tree_plan(T.shape, K, "balanced")).iterate(3)
    np.testing.assert_allclose(e_ch, e_dp, rtol=1e-12)
    np.testing.assert_allclose(e_bal, e_dp, rtol=1e-12)


CASES = [
    # (L, K, storage, compute, normwise bar reported beside the element-wise check)
    ((64, 64, 64), (8, 8, 8), "f64", "fp64", 1e-10),
    ((24, 20, 16, 12), (4, 5, 3, 6), "f32", "fp32", 1e-5),
    ((30, 7, 9, 5), (3, 2, 4, 2), "f32", "fp32", 1e-5),
    ((12, 11, 10, 9, 8), (3, 3, 2, 2, 4), "f32", "fp32", 1e-5),
    ((16, 12, 10, 8, 6, 4), (4, 4, 3, 3, 2, 2), "f32", "fp32", 1e-5),
    ((20, 20, 20, 20, 20), (4, 4, 4, 4, 4), "bf16", "fp32", 1e-5),
    ((20, 20, 20, 20, 20), (4, 4, 4, 4, 4), "f16", "fp32", 1e-5),
    ((24, 20, 16, 12), (4, 5, 3, 6), "f16", "fp32", 1e-5),
    ((40, 33, 17), (6, 5, 7), "f64", "fp64", 1e-10),
    # reduced precision, bounds per leaf against the exact chain: bf16x3 1e-4;
    # BF16 1.5e-2 for up to five rounded TTMs on the path to a leaf
    ((24, 20, 16, 12), (4, 5, 3, 6), "f32", "bf16x3", 1e-4),
    ((12, 11, 10, 9, 8), (3, 3, 2, 2, 4), "f32", "bf16", 1.5e-2),
    ((16, 12, 10, 8, 6, 4), (4, 4, 3, 3, 2, 2), "f32", "bf16", 1.5e-2),
    ((20, 20, 20, 20, 20), (4, 4, 4, 4, 4), "bf16", "bf16", 1.5e-2),
    ((20, 20, 20, 20, 20), (4, 4, 4, 4, 4), "bf16", "bf16x3", 1e-4),
    ((64, 48, 40, 32), (8, 12, 4, 16), "f32", "bf16", 1.5e-2),
    ((64, 48, 40, 32), (8, 12, 4, 16), "f32", "bf16x3", 1e-4),
]


@pytest.mark.parametrize("L,K,dtype,compute,tol", CASES)
@pytest.mark.parametrize("kind", ["dp", "chain", "balanced"])
def test_tree_leaves_equal_naive_chain(L, K, dtype, compute, tol, kind):
    print(f"leaves L={L} K={K} {dtype}/{compute} {kind}", flush=True)
    T, _ = synth.planted(L, K, noise=1e-2, noise_kind="rel", dtype=dtype, cfg=70, idx=len(L))
    T64 = O.as_f64(T, dtype)
    g = np.random.default_rng(17)
    F = [np.linalg.qr(g.standard_normal((L[n], K[n])))[0] for n in range(len(L))]
    if compute != "fp64":
        F = [f.astype(np.float32).astype(np.float64) for f in F]  # both sides see the same F
    ctx = tk.hooi_init(_device_T(T, dtype), K, compute=compute, F0=F,
                       plan=tk.ttm_tree_plan(L, K, kind))
    ctx.tree_pass()
    core = O.new_core(T64, F)
    g2 = float(np.sum(core * core))
    for n in range(len(L)):
        Y = O.chain_except(T64, F, n)
        Ya = abs_chain(T64, F, n)
        etol = chain_tol([L[j] for j in range(len(L)) if j != n], compute,
                         bf16_input=dtype == "bf16")
        if compute == "fp64":
            etol *= 2  # the oracle rounds in FP64 too
        leaf = ctx.leaf(n)
        assert_elementwise(leaf, Y, Ya, etol, f"leaf {n} {kind} {dtype}/{compute}")
        assert rel_err(leaf, Y) < tol, n
        S = ctx.gram(n)
        C = Y.size // L[n]
        assert_elementwise(S, O.gram(Y, n), O.gram(Ya, n), 2 * etol + 2 * (C + 2) * 2.0 ** -53,
                           f"gram {n} {kind} {dtype}/{compute}")
        # ||G||^2 = trace(F_n^T S_n F_n) for every n
        assert abs(np.trace(F[n].T @ S @ F[n]) - g2) < 4 * tol * g2


def test_fp32_iterations_match_oracle():
    L, K = (30, 28, 26, 24), (5, 4, 6, 3)
    T, _ = synth.planted(L, K, noise=1e-3, noise_kind="rel", dtype="f32", cfg=71)
    T64 = T.astype(np.float64)
    ctx = tk.hooi_init(_device_T(T, "f32"), K, compute="fp32")
    errs = ctx.iterate(4)
    Fo, Go, errs_o = O.hooi(T64, K, 4)
    # the identity error is sqrt(1 - ||G||^2/||T||^2): FP32 TTMs perturb ||G||^2 by ~1e-7
    # relative, i.e. err^2 by 1e-7/err^2 relative
    for e, eo in zip(errs, errs_o):
        assert abs(e * e - eo * eo) < 5e-7
    for n in range(4):
        assert subspace_dist(ctx.factor(n), Fo[n]) < 1e-4
    assert abs(ctx.error_explicit() - errs_o[-1]) < 1e-3 * errs_o[-1]


def test_f16_storage_iterations_match_oracle():
    """IEEE half storage, FP32 compute: the oracle runs in FP64 on the same
    stored values (exact in FP32), so the FP32 bars of the FP32-storage test
    hold."""
    L, K = (30, 28, 26, 24), (5, 4, 6, 3)
    T, _ = synth.planted(L, K, noise=1e-3, noise_kind="rel", dtype="f16", cfg=71)
    T64 = O.as_f64(T, "f16")
    print("f16 storage, fp32 HOOI 30x28x26x24", flush=True)
    ctx = tk.hooi_init(_device_T(T, "f16"), K, compute="fp32")
    errs = ctx.iterate(4)
    Fo, Go, errs_o = O.hooi(T64, K, 4)
    print(f"errors gpu {errs} oracle {errs_o}", flush=True)
    for e, eo in zip(errs, errs_o):
        assert abs(e * e - eo * eo) < 5e-7
    for n in range(4):
        assert subspace_dist(ctx.factor(n), Fo[n]) < 1e-4
    assert abs(ctx.error_explicit() - errs_o[-1]) < 1e-3 * errs_o[-1]


@pytest.mark.parametrize("compute", ["bf16", "bf16x3"])
def test_f16_storage_rejects_bf16_compute(compute):
    T, _ = synth.planted((8, 8, 8), (2, 2, 2), noise=0.0, dtype="f16", cfg=71)
    with pytest.raises(tk.TuckerError):
        tk.hooi_init(_device_T(T, "f16"), (2, 2, 2), compute=compute)
    with pytest.raises(tk.TuckerError):
        tk.hooi_init(_device_T(T, "f16"), (2, 2, 2), compute=compute, init="sthosvd")


@pytest.mark.parametrize("compute", ["bf16", "bf16x3"])
def test_reduced_precision_iterations_match_oracle(compute):
    """BF16-stored planted tensor (five modes), HOOI in BF16 / bf16x3 against
    the FP64 oracle on the same stored values.  The error is stationary in
    the factors, so factor perturbations enter it to second order: the
    relative error of the Tucker error is bounded by 1e-3."""
    L, K = (24, 24, 24, 24, 24), (4, 4, 4, 4, 4)
    T, _ = synth.planted(L, K, noise=1e-2, noise_kind="rel", dtype="bf16", cfg=72)
    T64 = O.as_f64(T, "bf16")
    print(f"bf16 storage, {compute} HOOI 24^5", flush=True)
    ctx = tk.hooi_init(_device_T(T, "bf16"), K, compute=compute)
    errs = ctx.iterate(3)
    Fo, Go, errs_o = O.hooi(T64, K, 3)
    print(f"errors gpu {errs} oracle {errs_o}", flush=True)
    dists = [subspace_dist(ctx.factor(n), Fo[n]) for n in range(5)]
    print(f"subspace distances {dists}", flush=True)
    for e, eo in zip(errs, errs_o):
        assert abs(e - eo) < 1e-3 * eo
    assert abs(ctx.error_explicit() - errs_o[-1]) < 1e-3 * errs_o[-1]
    assert max(dists) < (1e-1 if compute == "bf16" else 1e-3)


@pytest.mark.parametrize("L,K", [((64, 20, 12, 10), (6, 4, 3, 3)),
                                 ((64, 48, 40, 32, 24, 16)[:4], (8, 8, 6, 6))])
def test_modes_of_different_block_widths(L, K):
    """Modes with different eigensolver block widths (p = L_n up to 64), so the
    batched HOSVD launch runs every job at the widest width with V and W in
    the global work area: HOSVD and three invocations against the oracle."""
    T, _ = synth.planted(L, K, noise=1e-3, noise_kind="rel", dtype="f64", cfg=73)
    print(f"block widths L={L} K={K}", flush=True)
    ctx = tk.hooi_init(_device_T(T, "f64"), K, compute="fp64")
    F0 = O.hosvd(T, K)
    for n in range(len(L)):
        assert subspace_dist(ctx.factor(n), F0[n]) < 1e-9
    errs = ctx.iterate(3)
    Fo, Go, errs_o = O.hooi(T, K, 3)
    # identity error: ||G||^2 in FP64 moves e^2 by ~1e-16 ||T||^2-relative sums
    for e, eo in zip(errs, errs_o):
        assert abs(e * e - eo * eo) < 1e-13
    for n in range(len(L)):
        assert subspace_dist(ctx.factor(n), Fo[n]) < 1e-9


def test_checkpoint_resume_is_exact_and_runs_are_deterministic():
    T, info = synth.workload("planted_64x64x64_r8_f64")
    K = info["K"]
    Td = _device_T(T, "f64")
    a = tk.hooi_init(Td, K, compute="fp64")
    e_all = a.iterate(4)
    b = tk.hooi_init(Td, K, compute="fp64")
    e1 = b.iterate(2)
    Fmid = b.factors()
    c = tk.hooi_init(Td, K, compute="fp64", F0=Fmid)
    e2 = c.iterate(2)
    # factors are bitwise identical; the error of the iterate at the resume point
    # comes from the direct core chain instead of the folded core (another
    # summation order), so errors agree to rounding of 1 - ||G||^2/||T||^2
    for n in range(3):
        np.testing.assert_array_equal(c.factor(n), a.factor(n))
    np.testing.assert_allclose(np.array(e1 + e2), np.array(e_all), rtol=1e-12)
    d = tk.hooi_init(Td, K, compute="fp64")
    np.testing.assert_array_equal(np.array(d.iterate(4)), np.array(e_all))


def test_bad_factors_rejected():
    T, info = synth.workload("planted_64x64x64_r8_f64")
    K = info["K"]
    F = [np.zeros((64, 8)) for _ in range(3)]
    F[1][3, 2] = np.nan
    with pytest.raises(tk.TuckerError) as e:
        tk.hooi_init(_device_T(T, "f64"), K, compute="fp64", F0=F)
    assert e.value.code == tk.TK_ENUMERIC


def test_gapless_gaussian_tensor_matches_oracle():
    """A pure Gaussian 96x80x72 tensor with K = 8 per mode: no planted gap,
    modes above 64 (subspace eigensolves), so a solve may not converge and
    falls back to the gap-free solver instead of failing.  FP64 HOSVD and
    three invocations against the oracle: errors 1e-10 relative, subspaces
    1e-6 (the spectra have small gaps at K)."""
    L, K = (96, 80, 72), (8, 8, 8)
    g = np.random.default_rng(96)
    T = g.standard_normal(L)
    print("gapless gaussian 96x80x72 K=8 fp64", flush=True)
    ctx = tk.hooi_init(_device_T(T, "f64"), K, compute="fp64")
    F0 = O.hosvd(T, K)
    for n in range(3):
        assert subspace_dist(ctx.factor(n), F0[n]) < 1e-6
    errs = ctx.iterate(3)
    Fo, Go, errs_o = O.hooi(T, K, 3, F0=F0)
    print(f"errors gpu {errs} oracle {errs_o}", flush=True)
    np.testing.assert_allclose(errs, errs_o, rtol=1e-10)
    assert abs(ctx.error_explicit() - errs_o[-1]) < 1e-10 * errs_o[-1]
    for n in range(3):
        assert subspace_dist(ctx.factor(n), Fo[n]) < 1e-6


@pytest.mark.parametrize("dtype,compute", [("f64", "fp64"), ("f32", "fp32")])
def test_ranks_above_subspace_block_limit(dtype, compute):
    """K_0 = 60 > 48: that mode's factors come from the gap-free solver
    (Householder tridiagonalisation + QL) at every solve.  HOSVD and two
    invocations against the oracle."""
    L, K = (128, 70, 40), (60, 20, 12)
    T, _ = synth.planted(L, K, noise=1e-2, noise_kind="rel", dtype=dtype, cfg=74)
    T64 = O.as_f64(T, dtype)
    print(f"K above the block limit: L={L} K={K} {dtype}/{compute}", flush=True)
    ctx = tk.hooi_init(_device_T(T, dtype), K, compute=compute)
    F0 = O.hosvd(T64, K)
    for n in range(3):
        assert subspace_dist(ctx.factor(n), F0[n]) < 1e-8
    errs = ctx.iterate(2)
    Fo, Go, errs_o = O.hooi(T64, K, 2, F0=F0)
    print(f"errors gpu {errs} oracle {errs_o}", flush=True)
    tol = 1e-10 if compute == "fp64" else 1e-3
    np.testing.assert_allclose(errs, errs_o, rtol=tol)
    for n in range(3):
        assert subspace_dist(ctx.factor(n), Fo[n]) < (1e-8 if compute == "fp64" else 1e-4)


@pytest.mark.parametrize("L,K,dtype,compute,order", [
    ((40, 33, 17), (6, 5, 7), "f64", "fp64", None),
    ((30, 28, 26, 24), (5, 4, 6, 3), "f64", "fp64", (2, 0, 3, 1)),
    ((48, 40, 36, 32), (6, 5, 4, 4), "f32", "fp32", None),
    ((36, 30, 28, 22), (5, 6, 4, 3), "f16", "fp32", (1, 3, 0, 2)),
    ((24, 20, 16, 12, 10), (4, 5, 3, 6, 2), "bf16", "bf16x3", (4, 3, 2, 1, 0)),
])
def test_sthosvd_start_matches_oracle(L, K, dtype, compute, order):
    """STHOSVD start (sequential truncation) against the oracle's: factor
    subspaces, and the decomposition's error equal to the oracle's (whose
    square is the sum of the energy the truncations discard).  FP64: 1e-10;
    FP32 truncations: subspaces 1e-5, errors 1e-4 relative (relative noise
    1e-2)."""
    T, _ = synth.planted(L, K, noise=1e-2, noise_kind="rel", dtype=dtype, cfg=75)
    T64 = O.as_f64(T, dtype)
    print(f"sthosvd L={L} K={K} {dtype}/{compute} order={order}", flush=True)
    ctx = tk.hooi_init(_device_T(T, dtype), K, compute=compute, init="sthosvd", order=order)
    Fo, Go, disc = O.sthosvd(T64, K, order=order)
    eo = O.rel_error_explicit(T64, Go, Fo)
    assert abs(eo * eo * float(np.sum(T64 * T64)) - sum(disc)) < 1e-10 * float(np.sum(T64 * T64))
    fp64 = compute == "fp64"
    for n in range(len(L)):
        assert subspace_dist(ctx.factor(n), Fo[n]) < (1e-10 if fp64 else 1e-5), n
    e_exp = ctx.error_explicit()
    assert abs(e_exp - eo) < (1e-10 if fp64 else 1e-4) * eo
    # HOOI from there agrees with the oracle's HOOI from its STHOSVD factors;
    # the two starts differ by rounding (~1e-12), which the first invocations
    # carry into the error to first order (it is stationary only at a fixed
    # point): 1e-8 in FP64
    errs = ctx.iterate(2)
    _, _, errs_o = O.hooi(T64, K, 2, F0=Fo)
    for e, ref in zip(errs, errs_o):
        assert abs(e - ref) < (1e-8 if fp64 else 1e-3) * ref


def test_sthosvd_rejects_bad_order():
    T, info = synth.workload("planted_64x64x64_r8_f64")
    with pytest.raises(tk.TuckerError) as e:
        tk.hooi_init(_device_T(T, "f64"), info["K"], compute="fp64", init="sthosvd",
                     order=(0, 0, 1))
    assert e.value.code == tk.TK_EINVAL
