"""Seeded synthetic inputs for the dense Tucker / HOOI path.

The inputs follow the recipe of the paper's benchmark (metadata-driven,
randomly filled tensors, Sec. 6.1) specialised to planted low-rank tensors:

    X = G x_1 U_1 x_2 U_2 ... x_N U_N,     T = X + noise,

with a Gaussian (or deterministic decaying) core G, orthonormal factors U_n
(Q of the reduced QR of an N(0,1) L_n x K_n matrix) and Gaussian noise that is
either absolute (std sigma) or relative (scaled to nu * ||X||_F).

This module is shared by the oracle and by the GPU path's tests and benchmark.
It only *produces* tensors: it holds none of the method's arithmetic (no TTM
tree, no Gram/eigen step, no HOOI).  The planted tensor is assembled with
numpy.tensordot, a library contraction used purely as a data generator.

Every draw is seeded: numpy Generator(Philox(SeedSequence([17070559, cfg, i]))).
Large tensors are filled slab by slab with child seeds so that the result does
not depend on the number of worker threads.
"""
from __future__ import annotations

import concurrent.futures as _cf
import math
import os
import threading

import numpy as np

SEED_ROOT = 17070559

# BLAS and LAPACK calls (QR, tensordot, dot) are serialised: concurrent calls
# into the threaded BLAS from several Python threads have produced wrong
# results, and batch_tensors draws tensors on a thread pool.
_BLAS = threading.RLock()

# Workload table: each entry names one synthetic workload by its sizes.
WORKLOADS = {
    # 3-mode FP64 64^3, ranks 8, absolute N(0, 1e-3) noise
    "planted_64x64x64_r8_f64": dict(cfg=1, L=(64, 64, 64), K=(8, 8, 8),
                                    noise=1e-3, noise_kind="abs", core="normal",
                                    dtype="f64"),
    # 4-mode FP32 200^4, ranks 20, 1e-3 relative noise
    "planted_200x200x200x200_r20_f32": dict(cfg=2, L=(200,) * 4, K=(20,) * 4,
                                            noise=1e-3, noise_kind="rel",
                                            core="normal", dtype="f32"),
    # 5-mode 80^5 stored BF16, ranks 10, 1e-2 relative noise
    "planted_80x80x80x80x80_r10_bf16": dict(cfg=3, L=(80,) * 5, K=(10,) * 5,
                                            noise=1e-2, noise_kind="rel",
                                            core="normal", dtype="bf16"),
    # 6-mode FP32, ranks (8,8,6,6,4,4), core 1/(i1+...+i6), 1e-3 relative noise
    "planted_64x48x40x32x24x16_f32": dict(cfg=6, L=(64, 48, 40, 32, 24, 16),
                                          K=(8, 8, 6, 6, 4, 4), noise=1e-3,
                                          noise_kind="rel", core="decay",
                                          dtype="f32"),
}


# Real-tensor metadata (Sec. 6.1, table of real tensors): dimension lengths
# and core lengths.  The paper fills these tensors with random data.
REAL_TENSORS = {
    "HCCI": ((672, 672, 627, 16), (279, 279, 153, 14)),
    "TJLR": ((460, 700, 360, 16, 4), (306, 232, 239, 16, 4)),
    "SP": ((500, 500, 500, 11, 10), (81, 129, 127, 7, 6)),
}


def real_tensor_device(name: str, device, cfg: int = 7):
    """The real-tensor shape `name` filled with uniform [0, 1) FP32 values on
    a torch device, drawn by torch's generator for that device seeded from
    (SEED_ROOT, cfg, the shape's index).  4.5e9 to 1.4e10 elements: drawn
    where it is used; parity checks read slices back from the device."""
    import torch
    L, _ = REAL_TENSORS[name]
    g = torch.Generator(device=device)
    g.manual_seed(SEED_ROOT * 1000 + cfg * 10 + list(REAL_TENSORS).index(name))
    return torch.rand(L, generator=g, device=device, dtype=torch.float32)


def generator(cfg: int, idx: int = 0, stream: int = 0) -> np.random.Generator:
    """Seeded Philox generator for workload `cfg`, tensor `idx`, sub-stream `stream`."""
    return np.random.Generator(np.random.Philox(
        np.random.SeedSequence([SEED_ROOT, int(cfg), int(idx), int(stream)])))


def orthonormal(g: np.random.Generator, L: int, K: int) -> np.ndarray:
    """Q factor of the reduced QR of an N(0,1) L x K matrix (float64)."""
    a = g.standard_normal((L, K))
    with _BLAS:
        q, _ = np.linalg.qr(a)
    return q


def core_tensor(g: np.random.Generator, K, kind: str) -> np.ndarray:
    """Planted core: N(0,1) entries, or G[i] = 1/(i_1+...+i_N) with 1-based i."""
    K = tuple(int(k) for k in K)
    if kind == "normal":
        return g.standard_normal(K)
    if kind == "decay":
        grids = np.meshgrid(*[np.arange(1, k + 1, dtype=np.float64) for k in K],
                            indexing="ij")
        return 1.0 / sum(grids)
    raise ValueError(f"unknown core kind {kind!r}")


def _assemble(G: np.ndarray, U, dtype) -> np.ndarray:
    """X = G x_1 U_1 ... x_N U_N assembled with tensordot (data generation only)."""
    X = G.astype(dtype)
    N = X.ndim
    for n in range(N):
        # contract axis n of X with columns of U_n; tensordot puts the new axis last
        with _BLAS:
            X = np.tensordot(X, U[n].astype(dtype).T, axes=([n], [0]))
        X = np.moveaxis(X, -1, n)
    return np.ascontiguousarray(X)


def _fill_normal(out: np.ndarray, cfg: int, idx: int, stream: int,
                 slab_elems: int = 1 << 24) -> None:
    """Fill a flat float32/float64 array with N(0,1), slab-seeded (thread-count independent)."""
    flat = out.reshape(-1)
    nslab = max(1, math.ceil(flat.size / slab_elems))

    def work(s):
        lo = s * slab_elems
        hi = min(flat.size, lo + slab_elems)
        g = generator(cfg, idx, 1000 + stream * 1_000_000 + s)
        g.standard_normal(out=flat[lo:hi], dtype=flat.dtype)

    if nslab == 1:
        work(0)
        return
    workers = min(16, os.cpu_count() or 1)
    with _cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(work, range(nslab)))


def round_to_bf16_bits(x: np.ndarray, chunk: int = 1 << 24) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even); return uint16 bits."""
    src = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    out = np.empty(src.size, dtype=np.uint16)

    def work(lo):
        u = src[lo:lo + chunk].view(np.uint32)
        bias = ((u >> np.uint32(16)) & np.uint32(1)) + np.uint32(0x7FFF)
        out[lo:lo + chunk] = (u + bias) >> np.uint32(16)

    starts = range(0, src.size, chunk)
    if src.size <= chunk:
        work(0)
    else:
        with _cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(work, starts))
    return out.reshape(np.shape(x))


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Exact upcast of bfloat16 bit patterns to float32."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def planted(L, K, *, noise: float, noise_kind: str = "rel", core: str = "normal",
            dtype: str = "f64", cfg: int = 0, idx: int = 0):
    """Planted Tucker tensor plus noise, rounded to the storage dtype.

    Returns (T_stored, info) where T_stored is float64/float32/float16 for
    "f64"/"f32"/"f16" and uint16 bfloat16 bit patterns for "bf16"; info holds the planted core
    and factors (float64) and the noise scale actually applied.
    """
    L = tuple(int(x) for x in L)
    K = tuple(int(x) for x in K)
    if len(L) != len(K):
        raise ValueError("L and K must have the same length")
    g = generator(cfg, idx, 0)
    G = core_tensor(g, K, core)
    U = [orthonormal(g, L[n], K[n]) for n in range(len(L))]
    work = np.float64 if dtype == "f64" else np.float32
    X = _assemble(G, U, work)
    if noise > 0.0:
        E = np.empty(X.shape, dtype=work)
        _fill_normal(E, cfg, idx, 0)
        if noise_kind == "abs":
            scale = float(noise)
        elif noise_kind == "rel":
            with _BLAS:
                nx = float(np.sqrt(np.dot(X.reshape(-1).astype(np.float64, copy=False),
                                          X.reshape(-1).astype(np.float64, copy=False)))) \
                    if X.size < (1 << 27) else _norm_chunked(X)
                ne = float(np.sqrt(np.dot(E.reshape(-1).astype(np.float64, copy=False),
                                          E.reshape(-1).astype(np.float64, copy=False)))) \
                    if E.size < (1 << 27) else _norm_chunked(E)
            scale = float(noise) * nx / ne
        else:
            raise ValueError(f"unknown noise kind {noise_kind!r}")
        _axpy_chunked(X, E, work(scale))
        del E
    else:
        scale = 0.0
    if dtype == "bf16":
        Ts = round_to_bf16_bits(X)
    elif dtype == "f16":
        Ts = X.astype(np.float16)  # IEEE round to nearest even
    elif dtype in ("f32", "f64"):
        Ts = X
    else:
        raise ValueError(f"unknown dtype {dtype!r}")
    return Ts, dict(core=G, factors=U, noise_scale=scale, L=L, K=K, dtype=dtype)


def _norm_chunked(X: np.ndarray, chunk: int = 1 << 25) -> float:
    flat = X.reshape(-1)
    acc = 0.0
    for lo in range(0, flat.size, chunk):
        c = flat[lo:lo + chunk].astype(np.float64)
        acc += float(np.dot(c, c))
    return math.sqrt(acc)


def _axpy_chunked(X: np.ndarray, E: np.ndarray, a, chunk: int = 1 << 25) -> None:
    fx = X.reshape(-1)
    fe = E.reshape(-1)
    for lo in range(0, fx.size, chunk):
        fe[lo:lo + chunk] *= a
        fx[lo:lo + chunk] += fe[lo:lo + chunk]


def workload(name: str, idx: int = 0):
    """Generate one named workload; returns (T_stored, info)."""
    w = WORKLOADS[name]
    return planted(w["L"], w["K"], noise=w["noise"], noise_kind=w["noise_kind"],
                   core=w["core"], dtype=w["dtype"], cfg=w["cfg"], idx=idx)


def batch_shapes(count: int = 512, cfg: int = 5, seed_idx: int = 0,
                 lmin: int = 32, lmax: int = 128, kmin: int = 4, kmax: int = 16):
    """Shapes of the uneven batch: each tensor is 3- or 4-mode (fair coin),
    mode sizes uniform in [lmin, lmax], ranks uniform in [kmin, kmax]
    (clipped to the mode size and to the product of the other ranks)."""
    g = generator(cfg, seed_idx, 7)
    out = []
    for _ in range(count):
        N = 3 if g.integers(0, 2) == 0 else 4
        L = [int(v) for v in g.integers(lmin, lmax + 1, size=N)]
        K = [int(v) for v in g.integers(kmin, kmax + 1, size=N)]
        K = [min(k, l) for k, l in zip(K, L)]
        for n in range(N):  # a rank above the product of the others is unattainable
            K[n] = min(K[n], int(np.prod([K[m] for m in range(N) if m != n])))
        out.append((tuple(L), tuple(K)))
    return out


def batch_tensors(shapes, *, noise: float = 1e-3, dtype: str = "f32", cfg: int = 5,
                  window: int = 32, workers: int = 0):
    """Yield (i, T_i) for the planted tensors of a batch, in order, drawing up
    to `window` tensors at a time on a thread pool (each draw is seeded by
    (cfg, i) alone, so the result does not depend on the pool)."""
    workers = workers or min(16, os.cpu_count() or 1)

    def one(i):
        L, K = shapes[i]
        T, _ = planted(L, K, noise=noise, noise_kind="rel", dtype=dtype, cfg=cfg, idx=i)
        return T

    with _cf.ThreadPoolExecutor(workers) as ex:
        for w0 in range(0, len(shapes), window):
            idx = list(range(w0, min(len(shapes), w0 + window)))
            for i, T in zip(idx, ex.map(one, idx)):
                yield i, T
