"""Kernel-level parity on the GPU: TTM node, Gram and FP64 eigensolver against
the FP64 oracle, called through the C ABI.

Every comparison is element-wise against the oracle's contraction of the
absolute values (tests/gpu_util.py states the bounds): a TTM with reduction
length L is within (L + 2) u of that magnitude bound (u = 2^-24 for FP32,
2^-53 for FP64; 3 L + 2 for FP32 compute on BF16 input, which sums three exact
products per term), and the reduced-precision modes add their operand
rounding.  The Gram from FP32/BF16 inputs is formed from exact FP64 products,
so its bound is (C + 2) 2^-53 for C columns."""
import numpy as np
import pytest

import synth
from oracle import hooi as O
from oracle import precision as P
from tests.gpu_util import (abs_gram, abs_ttm, assert_elementwise, subspace_dist,
                            to_dev, torch_dev, ttm_tol)

pytestmark = pytest.mark.gpu

tk = pytest.importorskip("paper_1707_05594_amd")

# (A, L, B, K) covering: B % 4 == 0 wide path with a ragged tail, B = 1, odd B,
# small B, A = 1, K = 1, K = L, K not a multiple of 4, K above one LDS chunk.
TTM_CASES = [
    (3, 37, 1000, 5),
    (1, 64, 4096, 20),
    (1000, 50, 1, 7),
    (37, 29, 7, 3),
    (64, 33, 12, 16),
    (5, 17, 20, 1),
    (4, 16, 64, 16),
    (2, 200, 200, 20),
    (9, 23, 40, 23),
    (3, 129, 33, 70),
    (777, 10, 1, 10),
    (1000, 64, 1, 20),   # row path (B = 1, L % 4 == 0)
    (257, 200, 1, 37),   # row path, K over several groups, ragged rows
    (5, 48, 1, 3),       # row path, tiny grid
    (300, 68, 1, 12),    # row tiles: short last column chunk, last wave partial
    (70, 4, 1, 5),       # row tiles: one four-column chunk
    (1, 36, 1, 2),       # row tiles: a single row
    (2000, 1000, 1, 8),  # row tiles: one K-group beside the tiles, two K-chunks
    (300, 2000, 1, 4),   # rows too long for the tiles: direct row loads
    (5, 1, 64, 3),       # small wide grid (split L): one row, three waves idle
    (1, 300, 32, 24),    # small wide grid: K over six chunks
    (200, 200, 400, 20), # small wide grid: 313 blocks of 256 columns
    (13201, 32, 20, 6),  # slab-aligned wide path: 80-byte runs, 12 slabs per wave, ragged A
    (1320, 40, 200, 20), # slab-aligned wide path: one 800-byte-run slab per wave
    (7, 50, 37, 12),     # 4-byte-load wide path: odd B, columns across a boundaries
    (300, 30, 1001, 20), # 4-byte-load wide path on a full grid, ragged last wave
]

# Large ranks (several K-chunks of the capped instance): the factor staged 64
# rows at a time, K-chunks of a tile as consecutive work items of one XCD.
LK_CASES = [
    (3, 700, 100, 232),   # 16-byte body, 12 groups x 5 chunks, last row chunk of 60
    (2, 672, 627, 153),   # 4-byte body (odd B), 8 groups x 5 chunks, ragged last tile
    (1000, 161, 14, 81),  # short runs (B < 32) through the 4-byte body, 3 chunks
    (50, 500, 64, 127),   # 16-byte body, 12 groups x 3 chunks (K = 127, ragged groups)
    (1, 460, 5345, 306),  # 4-byte body, 10 chunks, one a
    (7, 65, 1024, 96),    # 16-byte body, 2 chunks, a last row chunk of one row
]


# Short slabs (L <= 32; B = 1 or B < 32 off the wide path): a wave owns 64 / B
# whole slabs, contiguous input and output ranges staged through its LDS
# area.  Rows of 10, 11, 16 and 4 elements with K close to L (the real
# tensors' trailing modes), B = 6 and 13 (partial lane use), B = 31 (two
# slabs per wave), K = 32 (eight groups), ragged last waves and a single slab.
SHORT_CASES = [
    (1000, 10, 1, 6), (777, 11, 6, 7), (513, 16, 1, 14), (300, 4, 1, 4),
    (1001, 32, 3, 32), (65, 5, 31, 3), (129, 7, 13, 5), (1, 3, 1, 2),
]


@pytest.mark.parametrize("A,L,B,K", TTM_CASES + LK_CASES + SHORT_CASES)
def test_ttm_fp32(A, L, B, K):
    torch, dev = torch_dev()
    print(f"ttm fp32 A={A} L={L} B={B} K={K}", flush=True)
    g = np.random.default_rng(A * 1000 + L * 10 + K)
    X = g.standard_normal((A, L, B)).astype(np.float32)
    F = g.standard_normal((L, K)).astype(np.float32)
    out = torch.full((A, K, B), float("nan"), dtype=torch.float32, device=dev)
    tk.ttm(to_dev(X), A, L, B, to_dev(F), K, out)
    torch.cuda.synchronize()
    X64, F64 = X.astype(np.float64), F.astype(np.float64)
    ref = O.ttm(X64, F64.T, 1)
    assert_elementwise(out.cpu().numpy(), ref, abs_ttm(X64, F64.T, 1), ttm_tol(L, "fp32"),
                       f"ttm fp32 {A}x{L}x{B} K={K}")


@pytest.mark.parametrize("A,L,B,K", TTM_CASES[:6] + TTM_CASES[-13:] + LK_CASES + SHORT_CASES)
def test_ttm_bf16_storage_fp32_compute(A, L, B, K):
    torch, dev = torch_dev()
    print(f"ttm bf16 A={A} L={L} B={B} K={K}", flush=True)
    g = np.random.default_rng(7 + A + L + B + K)
    X = g.standard_normal((A, L, B)).astype(np.float32)
    Xb = synth.round_to_bf16_bits(X)
    F = g.standard_normal((L, K)).astype(np.float32)
    xt = torch.from_numpy(Xb.view(np.int16)).view(torch.bfloat16).to(dev)
    out = torch.empty((A, K, B), dtype=torch.float32, device=dev)
    tk.ttm(xt, A, L, B, to_dev(F), K, out)
    torch.cuda.synchronize()
    X64, F64 = O.as_f64(Xb, "bf16"), F.astype(np.float64)
    ref = O.ttm(X64, F64.T, 1)
    assert_elementwise(out.cpu().numpy(), ref, abs_ttm(X64, F64.T, 1),
                       ttm_tol(L, "fp32", bf16_input=True), f"ttm bf16->fp32 {A}x{L}x{B} K={K}")


@pytest.mark.parametrize("A,L,B,K", TTM_CASES[:6] + TTM_CASES[-13:] + LK_CASES + SHORT_CASES)
def test_ttm_f16_storage_fp32_compute(A, L, B, K):
    """IEEE half storage: every value is exact in FP32, so the FP32 kernels
    (converting on load) meet the FP32 bound on the stored values."""
    torch, dev = torch_dev()
    print(f"ttm f16 A={A} L={L} B={B} K={K}", flush=True)
    g = np.random.default_rng(11 + A + L + B + K)
    Xh = g.standard_normal((A, L, B)).astype(np.float16)
    F = g.standard_normal((L, K)).astype(np.float32)
    out = torch.full((A, K, B), float("nan"), dtype=torch.float32, device=dev)
    tk.ttm(torch.from_numpy(Xh).to(dev), A, L, B, to_dev(F), K, out)
    torch.cuda.synchronize()
    X64, F64 = O.as_f64(Xh, "f16"), F.astype(np.float64)
    ref = O.ttm(X64, F64.T, 1)
    assert_elementwise(out.cpu().numpy(), ref, abs_ttm(X64, F64.T, 1), ttm_tol(L, "fp32"),
                       f"ttm f16->fp32 {A}x{L}x{B} K={K}")


@pytest.mark.parametrize("compute", ["bf16", "bf16x3"])
def test_ttm_f16_storage_rejects_bf16_compute(compute):
    torch, dev = torch_dev()
    x = torch.zeros((4, 8, 4), dtype=torch.float16, device=dev)
    F = torch.zeros((8, 2), dtype=torch.float32, device=dev)
    out = torch.empty((4, 2, 4), dtype=torch.float32, device=dev)
    with pytest.raises(tk.TuckerError):
        tk.ttm(x, 4, 8, 4, F, 2, out, compute=compute)


def _bf16_mfma_path(A, L, B):
    """Nodes the BF16 kernels take: wide nodes whose 1024-column grid fills the
    chip (256 blocks), and rows with L % 4 == 0.  Others run FP32 kernels (the
    tile kernel, or the split-L wide kernel on small grids)."""
    wide = B % 4 == 0 and B >= 16 and (A * B + 1023) // 1024 >= 256
    return wide or (B == 1 and L % 4 == 0)


# Reduced precision.  On the BF16 kernels every product of two bfloat16 values
# is exact in FP32, so the result equals the float64 model of the mode
# (oracle.precision) up to FP32 accumulation of L (BF16) or 3 L (bf16x3)
# exact products.  Against the exact product the per-element bounds add the
# operand rounding: 2^-7 + 2^-16 for BF16 (one rounding of each operand,
# 2^-8 relative), 4 * 2^-16 for bf16x3 (2^-16 representation error per
# operand plus the dropped lo * lo product).


@pytest.mark.parametrize("A,L,B,K", TTM_CASES + [(2, 64, 4096, 48), (4, 2048, 16, 5),
                                                 (300, 400, 1, 44), (512, 16, 512, 20),
                                                 (3, 37, 100000, 5)])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("compute", ["bf16", "bf16x3"])
def test_ttm_reduced_precision(A, L, B, K, storage, compute):
    torch, dev = torch_dev()
    print(f"ttm {storage}/{compute} A={A} L={L} B={B} K={K}", flush=True)
    g = np.random.default_rng(23 + A + 3 * L + 5 * B + 7 * K)
    X = g.standard_normal((A, L, B)).astype(np.float32)
    F = g.standard_normal((L, K)).astype(np.float32)
    if storage == "bf16":
        Xb = synth.round_to_bf16_bits(X)
        xt = torch.from_numpy(Xb.view(np.int16)).view(torch.bfloat16).to(dev)
        X64 = O.as_f64(Xb, "bf16")
    else:
        xt = to_dev(X)
        X64 = X.astype(np.float64)
    out = torch.full((A, K, B), float("nan"), dtype=torch.float32, device=dev)
    tk.ttm(xt, A, L, B, to_dev(F), K, out, compute=compute)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    F64 = F.astype(np.float64)
    exact = O.ttm(X64, F64.T, 1)
    mag = abs_ttm(X64, F64.T, 1)
    tag = f"ttm {storage}/{compute} {A}x{L}x{B} K={K}"
    if _bf16_mfma_path(A, L, B):
        if compute == "bf16":
            model = P.ttm_bf16(X64, F.T, 1)
            tol = ttm_tol(L, "fp32")
        else:
            model = P.ttm_bf16x3(X64, F.T, 1, x_is_bf16=storage == "bf16")
            tol = ttm_tol(L, "fp32", bf16_input=True)
        # model terms are products of operands within 2^-8 of the exact ones
        assert_elementwise(got, model, mag, tol * (1 + 2.0 ** -6), tag + " vs model")
    else:
        assert_elementwise(got, exact, mag, ttm_tol(L, "fp32", bf16_input=storage == "bf16"),
                           tag + " (FP32 kernel)")
    assert_elementwise(got, exact, mag, ttm_tol(L, compute), tag + " vs exact")


@pytest.mark.parametrize("A,L,B,K", [(3, 37, 100, 5), (100, 64, 1, 8), (7, 20, 9, 20),
                                     (2, 64, 64, 33)])
def test_ttm_fp64(A, L, B, K):
    torch, dev = torch_dev()
    print(f"ttm fp64 A={A} L={L} B={B} K={K}", flush=True)
    g = np.random.default_rng(11 + A + K)
    X = g.standard_normal((A, L, B))
    F = g.standard_normal((L, K))
    out = torch.empty((A, K, B), dtype=torch.float64, device=dev)
    tk.ttm(to_dev(X), A, L, B, to_dev(F), K, out, compute="fp64")
    torch.cuda.synchronize()
    # both sides round in FP64: twice the bound of one
    assert_elementwise(out.cpu().numpy(), O.ttm(X, F.T, 1), abs_ttm(X, F.T, 1),
                       2 * ttm_tol(L, "fp64"), f"ttm fp64 {A}x{L}x{B} K={K}")


def test_ttm_identity_factor_copies_input():
    torch, dev = torch_dev()
    g = np.random.default_rng(5)
    X = g.standard_normal((6, 12, 8)).astype(np.float32)
    out = torch.empty((6, 12, 8), dtype=torch.float32, device=dev)
    tk.ttm(to_dev(X), 6, 12, 8, to_dev(np.eye(12, dtype=np.float32)), 12, out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), X)


@pytest.mark.parametrize("A,L,B,dtype", [(1, 200, 8000, "f32"), (400, 200, 20, "f32"),
                                         (8000, 200, 1, "f32"), (3, 70, 13, "f64"),
                                         (16, 130, 16, "f32"), (5, 64, 33, "bf16"),
                                         # few rows over many columns; one row; one
                                         # valid row in the last 64-row tile with a
                                         # ragged last column chunk; B = 1 from BF16
                                         (200, 20, 400, "f32"), (2, 1, 50, "f32"),
                                         (1, 65, 12345, "f32"), (7, 17, 1, "bf16"),
                                         (300, 33, 1, "f64"), (5, 64, 33, "f16"),
                                         (1, 130, 999, "f16")])
def test_gram(A, L, B, dtype):
    torch, dev = torch_dev()
    print(f"gram A={A} L={L} B={B} {dtype}", flush=True)
    g = np.random.default_rng(A + L + B)
    Y = g.standard_normal((A, L, B))
    if dtype == "f32":
        Yd = to_dev(Y.astype(np.float32))
        Y64 = Y.astype(np.float32).astype(np.float64)
    elif dtype == "bf16":
        bits = synth.round_to_bf16_bits(Y.astype(np.float32))
        Yd = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).to(dev)
        Y64 = O.as_f64(bits, "bf16")
    elif dtype == "f16":
        Yh = Y.astype(np.float16)
        Yd = torch.from_numpy(Yh).to(dev)
        Y64 = O.as_f64(Yh, "f16")
    else:
        Yd = to_dev(Y)
        Y64 = Y
    S = torch.empty((L, L), dtype=torch.float64, device=dev)
    tk.gram(Yd, A, L, B, S)
    torch.cuda.synchronize()
    Sh = S.cpu().numpy()
    # both sides round in FP64: twice the bound of one
    assert_elementwise(Sh, O.gram(Y64, 1), abs_gram(Y64, 1), 2 * (A * B + 2) * 2.0 ** -53,
                       f"gram {A}x{L}x{B} {dtype}")
    np.testing.assert_array_equal(Sh, Sh.T)
    # deterministic: a second run gives identical bits
    S2 = torch.empty_like(S)
    tk.gram(Yd, A, L, B, S2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(S2.cpu().numpy(), Sh)


def _spd_with_gap(g, L, K, gap=1e6):
    Q, _ = np.linalg.qr(g.standard_normal((L, L)))
    w = np.concatenate([np.sort(g.uniform(1.0, 3.0, K))[::-1] * gap,
                        np.sort(g.uniform(0.0, 1.0, L - K))[::-1]])
    return (Q * w) @ Q.T


@pytest.mark.parametrize("L,K,warm", [(40, 5, False), (64, 8, False), (200, 20, False),
                                      (200, 20, True), (80, 10, True), (128, 16, False),
                                      (33, 33, False), (7, 1, False)])
def test_eig_leading(L, K, warm):
    torch, dev = torch_dev()
    print(f"eig L={L} K={K} warm={warm}", flush=True)
    g = np.random.default_rng(L * 3 + K)
    S = np.stack([_spd_with_gap(g, L, K) for _ in range(3)])
    V0 = None
    if warm:
        V0 = np.stack([np.linalg.qr(O.leading_eigvecs(s, K)[0] +
                                    1e-3 * g.standard_normal((L, K)))[0] for s in S])
    F, ev = tk.eig_leading(to_dev(S), K, V0=to_dev(V0) if V0 is not None else None)
    torch.cuda.synchronize()
    F = F.cpu().numpy()
    ev = ev.cpu().numpy()
    for m in range(3):
        Fr, wr = O.leading_eigvecs(S[m], K)
        np.testing.assert_allclose(ev[m], wr, rtol=1e-12)
        nS = np.linalg.norm(S[m], 2)
        assert np.linalg.norm(S[m] @ F[m] - F[m] * ev[m]) <= 1e-11 * nS
        assert np.linalg.norm(F[m].T @ F[m] - np.eye(K)) <= 1e-13
        assert subspace_dist(F[m], Fr) < 1e-10
        # eigenvalues are distinct: the sign rule makes the vectors unique
        assert np.abs(F[m] - Fr).max() < 1e-9


def test_eig_full_jacobi_random_small():
    # L <= 48 runs a full Jacobi: no gap needed
    torch, dev = torch_dev()
    g = np.random.default_rng(3)
    M = g.standard_normal((2, 30, 30))
    S = np.einsum("mij,mkj->mik", M, M)
    F, ev = tk.eig_leading(to_dev(S), 30)
    torch.cuda.synchronize()
    for m in range(2):
        w = np.linalg.eigvalsh(S[m])[::-1]
        np.testing.assert_allclose(ev.cpu().numpy()[m], w, rtol=1e-11, atol=1e-11 * w[0])


@pytest.mark.parametrize("L,K", [(64, 8), (56, 6), (49, 4)])
def test_eig_flat_trailing_spectrum(L, K):
    """Up to L = 64 every solve is a full Jacobi decomposition: exact even when
    the K-th eigenvalue sits in a nearly flat cluster (relative spacing ~1e-5),
    as for a planted core of lower numerical rank than K plus isotropic noise."""
    torch, dev = torch_dev()
    print(f"eig flat spectrum L={L} K={K}", flush=True)
    g = np.random.default_rng(L + 100 * K)
    S = []
    for _ in range(2):
        Q, _ = np.linalg.qr(g.standard_normal((L, L)))
        w = np.concatenate([[4e6, 2e5, 3e3], 1.0 + 1e-3 * g.uniform(0, 1, L - 3)])
        S.append((Q * w) @ Q.T)
    S = np.stack(S)
    for V0 in (None, np.stack([np.linalg.qr(g.standard_normal((L, K)))[0] for _ in range(2)])):
        F, ev = tk.eig_leading(to_dev(S), K, V0=to_dev(V0) if V0 is not None else None)
        torch.cuda.synchronize()
        F, ev = F.cpu().numpy(), ev.cpu().numpy()
        for m in range(2):
            wr = np.linalg.eigvalsh(S[m])[::-1][:K]
            np.testing.assert_allclose(ev[m], wr, rtol=1e-12, atol=1e-12 * wr[0])
            assert np.linalg.norm(S[m] @ F[m] - F[m] * ev[m]) <= 1e-11 * wr[0]
            assert np.linalg.norm(F[m].T @ F[m] - np.eye(K)) <= 1e-13


def test_fp32_compute_on_bf16_input_reproduces_24_bit_factors():
    """FP32 compute on BF16 input runs BF16 MFMAs with the factor split into
    three bfloat16 terms, which together hold all 24 bits of an FP32 entry.
    With f = 1 + 2^-10 + 2^-20 (its third term 2^-20 is nonzero) and an
    all-ones input, every output is 8 f exactly (all partial sums k f fit in
    24 bits); a two-term split would lose 8 * 2^-20.  The grid (262144 columns
    of L = 8) is wide enough for the split path."""
    torch, dev = torch_dev()
    A, L, B, K = 1, 8, 262144, 4
    ones = torch.ones((A, L, B), dtype=torch.bfloat16, device=dev)
    f = np.float32(1.0 + 2.0 ** -10 + 2.0 ** -20)
    F = np.full((L, K), f, dtype=np.float32)
    out = torch.empty((A, K, B), dtype=torch.float32, device=dev)
    tk.ttm(ones, A, L, B, to_dev(F), K, out)
    torch.cuda.synchronize()
    expect = np.float32(8.0 * float(f))
    assert float(expect) == 8.0 * float(f)  # exact in FP32
    np.testing.assert_array_equal(out.cpu().numpy(), np.full((A, K, B), expect, np.float32))


def _random_gram(g, L, C):
    """Gram of an L x C unfolding of a randomly filled tensor (Sec. 6.1 fills
    its benchmark tensors with random values): a Wishart-like spectrum with no
    planted gap anywhere."""
    Y = g.standard_normal((L, C))
    return Y @ Y.T


def _check_eig(S, F, ev, K, tag):
    """Eigenvalues within 1e-12 of the largest (absolute accuracy of a
    backward-stable solver), residual ||S F - F diag(ev)|| <= 1e-11 ||S||,
    orthonormality 1e-12, and each vector against eigh's, sign rule applied,
    within 1e-12 ||S|| / gap_j (its perturbation bound, gap_j = distance of
    eigenvalue j to the rest of the spectrum)."""
    w, V = np.linalg.eigh(S)
    order = np.argsort(-w, kind="stable")
    Fr = O.sign_rule(V[:, order[:K]])
    wr = w[order]
    nS = float(wr[0]) if wr[0] > 0 else 1.0
    np.testing.assert_allclose(ev, wr[:K], rtol=0, atol=1e-12 * nS, err_msg=tag)
    assert np.linalg.norm(S @ F - F * ev) <= 1e-11 * nS, tag
    assert np.abs(F.T @ F - np.eye(K)).max() <= 1e-12, tag
    for j in range(K):
        gap = min([abs(wr[j] - wr[i]) for i in range(len(wr)) if i != j] or [nS])
        if gap > 1e-6 * nS:
            err = np.abs(F[:, j] - Fr[:, j]).max()
            assert err <= 1e-12 * nS / gap + 1e-13, (tag, j, err, gap / nS)


@pytest.mark.parametrize("L,ratio", [(1, 1.0), (2, 1.0), (3, 1.5), (65, 1.25), (100, 1.25),
                                     (200, 2.0), (400, 1.25), (672, 1.25)])
def test_eig_full_random_gram(L, ratio):
    """The gap-free solver (tridiagonalisation + implicit QL) on Grams of
    randomly filled unfoldings with K = L / ratio (the paper's benchmark
    ranks, Sec. 6.1), against numpy.linalg.eigh."""
    torch, dev = torch_dev()
    K = max(1, int(round(L / ratio)))
    print(f"eig_full L={L} K={K}", flush=True)
    g = np.random.default_rng(L + 7)
    count = 2 if L <= 200 else 1
    S = np.stack([_random_gram(g, L, 2 * L + 3) for _ in range(count)])
    F, ev = tk.eig_full(to_dev(S), K)
    torch.cuda.synchronize()
    F, ev = F.cpu().numpy(), ev.cpu().numpy()
    for m in range(count):
        _check_eig(S[m], F[m], ev[m], K, f"L={L} K={K} m={m}")


@pytest.mark.parametrize("L,K", [(96, 8), (200, 20), (130, 48), (150, 100)])
def test_eig_leading_without_gap(L, K):
    """tk_eig_leading on matrices whose K-th eigenvalue sits in a nearly flat
    cluster (relative spacing 1e-6) with L > 64: subspace iteration cannot
    converge there and hands the matrix to the gap-free solver (and K > 48
    goes there directly); warm starts included.  The cluster makes single
    vectors undefined, so vectors are checked by residual and orthonormality
    and the K-dimensional subspace is compared only through the residual."""
    torch, dev = torch_dev()
    print(f"eig without gap L={L} K={K}", flush=True)
    g = np.random.default_rng(L * 5 + K)
    S = []
    for _ in range(2):
        Q, _ = np.linalg.qr(g.standard_normal((L, L)))
        top = np.sort(g.uniform(10.0, 100.0, K // 2))[::-1]
        w = np.concatenate([top, 1.0 + 1e-6 * g.uniform(0, 1, L - K // 2)])
        S.append((Q * w) @ Q.T)
    S = np.stack(S)
    starts = [None]
    if K <= 48:
        starts.append(np.stack([np.linalg.qr(g.standard_normal((L, K)))[0] for _ in range(2)]))
    for V0 in starts:
        F, ev = tk.eig_leading(to_dev(S), K, V0=to_dev(V0) if V0 is not None else None)
        torch.cuda.synchronize()
        F, ev = F.cpu().numpy(), ev.cpu().numpy()
        for m in range(2):
            wr = np.linalg.eigvalsh(S[m])[::-1][:K]
            np.testing.assert_allclose(ev[m], wr, rtol=0, atol=1e-12 * wr[0])
            assert np.linalg.norm(S[m] @ F[m] - F[m] * ev[m]) <= 1e-11 * wr[0]
            assert np.abs(F[m].T @ F[m] - np.eye(K)).max() <= 1e-12
            cols = np.arange(K)
            assert np.all(F[m][np.abs(F[m]).argmax(axis=0), cols] > 0)


# (A, Lp, M, Lq, B, Kp, Kq): the fused pass over both root children
PAIR_CASES = [
    (2, 37, 64, 200, 64, 20, 20),   # 200-row groups (last wave partly idle), K = 20 twice
    (3, 9, 240, 67, 12, 7, 13),     # ragged rows and K, short runs of b
    (1, 24, 512, 256, 16, 20, 1),   # every lane busy, K_q = 1
    (4096, 2, 1, 1, 4, 1, 1),       # one row: L_q = 1 (K_q = 1), M = 1
    (1, 64, 40, 48, 400, 8, 12),    # A = 1, wide b
]


@pytest.mark.parametrize("A,Lp,M,Lq,B,Kp,Kq", PAIR_CASES)
def test_ttm_pair_fp32(A, Lp, M, Lq, B, Kp, Kq):
    """Both root TTMs from one pass: each output element-wise against the
    oracle's TTM of the same input along p and along q (bound (L + 2) 2^-24
    of the magnitude bound), and bitwise repeatable."""
    torch, dev = torch_dev()
    print(f"ttm pair A={A} Lp={Lp} M={M} Lq={Lq} B={B} Kp={Kp} Kq={Kq}", flush=True)
    g = np.random.default_rng(A + Lp + M + Lq + B + Kp + Kq)
    X = g.standard_normal((A, Lp, M, Lq, B)).astype(np.float32)
    Fp = g.standard_normal((Lp, Kp)).astype(np.float32)
    Fq = g.standard_normal((Lq, Kq)).astype(np.float32)
    xd = to_dev(X)
    op = torch.full((A, Kp, M, Lq, B), float("nan"), dtype=torch.float32, device=dev)
    oq = torch.full((A, Lp, M, Kq, B), float("nan"), dtype=torch.float32, device=dev)
    tk.ttm_pair(xd, A, Lp, M, Lq, B, to_dev(Fp), Kp, to_dev(Fq), Kq, op, oq)
    torch.cuda.synchronize()
    X64 = X.astype(np.float64)
    Fp64, Fq64 = Fp.astype(np.float64), Fq.astype(np.float64)
    gp, gq = op.cpu().numpy(), oq.cpu().numpy()
    assert_elementwise(gp, O.ttm(X64, Fp64.T, 1), abs_ttm(X64, Fp64.T, 1), ttm_tol(Lp, "fp32"),
                       "pair: mode p")
    assert_elementwise(gq, O.ttm(X64, Fq64.T, 3), abs_ttm(X64, Fq64.T, 3), ttm_tol(Lq, "fp32"),
                       "pair: mode q")
    op2, oq2 = torch.empty_like(op), torch.empty_like(oq)
    tk.ttm_pair(xd, A, Lp, M, Lq, B, to_dev(Fp), Kp, to_dev(Fq), Kq, op2, oq2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(op2.cpu().numpy(), gp)
    np.testing.assert_array_equal(oq2.cpu().numpy(), gq)


def test_ttm_pair_rejects_unsupported():
    torch, dev = torch_dev()
    X = torch.zeros((1, 4, 8, 4, 6), dtype=torch.float32, device=dev)
    F = torch.zeros((4, 2), dtype=torch.float32, device=dev)
    o = torch.zeros(1024, dtype=torch.float32, device=dev)
    with pytest.raises(tk.TuckerError) as e:  # B % 4 != 0 and too few tiles
        tk.ttm_pair(X, 1, 4, 8, 4, 6, F, 2, F, 2, o, o)
    assert e.value.code == tk.TK_EUNSUPPORTED


@pytest.mark.parametrize("A,Lp,Lq,Kp,Kq", [
    # small slabs staged whole in LDS (the six-mode tensor's root pair)
    (4096, 24, 16, 4, 4), (5000, 12, 20, 7, 3), (4099, 8, 2, 8, 1), (9000, 1, 4, 1, 4),
    # large slabs streamed in row chunks: the 200^4 pair (ragged last chunk of
    # 8 rows), Lq = 256 with a ragged rank group, waves past Lq, a chunk
    # larger than the slab, two slabs per block with a ragged last block
    (300, 200, 200, 20, 20), (17, 300, 256, 17, 20), (40, 37, 132, 13, 7), (9, 5, 4, 3, 2),
    (20001, 12, 40, 5, 9)])
def test_ttm_pair_trailing_modes(A, Lp, Lq, Kp, Kq):
    """The pair kernels for the two trailing modes (slabs of Lp x Lq staged
    whole in LDS; or streamed through LDS in row chunks for large slabs and
    ranks up to 20): both outputs element-wise against the oracle, including
    ragged last chunks and blocks."""
    torch, dev = torch_dev()
    print(f"ttm pair (trailing) A={A} Lp={Lp} Lq={Lq} Kp={Kp} Kq={Kq}", flush=True)
    g = np.random.default_rng(A + Lp * Lq + Kp + Kq)
    X = g.standard_normal((A, Lp, Lq)).astype(np.float32)
    Fp = g.standard_normal((Lp, Kp)).astype(np.float32)
    Fq = g.standard_normal((Lq, Kq)).astype(np.float32)
    op = torch.full((A, Kp, Lq), float("nan"), dtype=torch.float32, device=dev)
    oq = torch.full((A, Lp, Kq), float("nan"), dtype=torch.float32, device=dev)
    tk.ttm_pair(to_dev(X), A, Lp, 1, Lq, 1, to_dev(Fp), Kp, to_dev(Fq), Kq, op, oq)
    torch.cuda.synchronize()
    X64, Fp64, Fq64 = X.astype(np.float64), Fp.astype(np.float64), Fq.astype(np.float64)
    assert_elementwise(op.cpu().numpy(), O.ttm(X64, Fp64.T, 1), abs_ttm(X64, Fp64.T, 1),
                       ttm_tol(Lp, "fp32"), "pair tail: mode p")
    assert_elementwise(oq.cpu().numpy(), O.ttm(X64, Fq64.T, 2), abs_ttm(X64, Fq64.T, 2),
                       ttm_tol(Lq, "fp32"), "pair tail: mode q")
