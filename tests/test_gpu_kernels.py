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


@pytest.mark.parametrize("A,L,B,K", TTM_CASES)
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


@pytest.mark.parametrize("A,L,B,K", TTM_CASES[:6] + TTM_CASES[-13:])
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
                                         (300, 33, 1, "f64")])
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
