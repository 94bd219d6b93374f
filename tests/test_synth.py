"""The seeded input generator: batch draws on a thread pool equal the serial
draws (each tensor is seeded by (cfg, index) alone), ranks of the uneven batch
are attainable, and relative noise has the requested norm."""
import math

import numpy as np

import synth


def test_threaded_batch_equals_serial_draws():
    shapes = synth.batch_shapes(24, cfg=5, seed_idx=9, lmin=16, lmax=72, kmin=2, kmax=8)
    for i, T in synth.batch_tensors(shapes, workers=16, window=12):
        d, _ = synth.planted(*shapes[i], noise=1e-3, noise_kind="rel", dtype="f32", cfg=5, idx=i)
        assert np.array_equal(T, d), i


def test_batch_ranks_attainable():
    for L, K in synth.batch_shapes(512, cfg=5, seed_idx=0):
        assert len(L) in (3, 4) and all(32 <= l <= 128 for l in L)
        for n in range(len(K)):
            assert 1 <= K[n] <= L[n]
            assert K[n] <= math.prod(K[m] for m in range(len(K)) if m != n)


def test_relative_noise_level():
    L, K = (20, 18, 16), (3, 4, 2)
    T, info = synth.planted(L, K, noise=1e-2, noise_kind="rel", dtype="f64", cfg=77)
    X, _ = synth.planted(L, K, noise=0.0, dtype="f64", cfg=77)
    rel = np.linalg.norm(T - X) / np.linalg.norm(X)
    assert abs(rel - 1e-2) < 1e-12
