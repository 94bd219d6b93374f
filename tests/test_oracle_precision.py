"""Pins of the reduced-precision TTM models (oracle.precision) on the CPU.

round_bf16 is checked against hand-worked values and against torch's
float32 -> bfloat16 cast (round to nearest even); the split and the bf16x3
product against their error bounds; the BF16 TTM against element-wise loops."""
import numpy as np
import pytest

from oracle import hooi as O
from oracle import precision as P


def test_round_bf16_hand_values():
    u = 2.0 ** -7  # spacing of bfloat16 values in [1, 2)
    cases = [
        (0.0, 0.0),
        (1.0, 1.0),
        (3.0, 3.0),
        (1 + u / 2, 1.0),                      # tie, 1.0 has an even significand
        (1 + 3 * u / 2, 1 + 2 * u),            # tie, rounds up to the even neighbour
        (1 + u / 2 + 2.0 ** -20, 1 + u),       # just above the tie
        (-(1 + u / 2 + 2.0 ** -20), -(1 + u)),
        (255.5, 256.0),                        # 8 significant bits: 255.5 -> 256 (tie to even)
        (2.0 ** -100 * 1.00390625, 2.0 ** -100),
        (1.9999, 2.0),
    ]
    for x, want in cases:
        assert P.round_bf16(x) == want, (x, P.round_bf16(x), want)


def test_round_bf16_matches_torch_cast():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(5)
    x = (g.standard_normal(200000) * np.exp(g.uniform(-30, 30, 200000))).astype(np.float32)
    # exact ties: bfloat16 values plus half a bfloat16 ulp
    base = P.round_bf16(g.standard_normal(2000).astype(np.float32))
    _, e = np.frexp(base)
    ties = (base + np.ldexp(1.0, e - 9)).astype(np.float32)
    x = np.concatenate([x, ties, -ties])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(P.round_bf16(x), want)


def test_split_bf16_bounds():
    g = np.random.default_rng(6)
    x = g.standard_normal(100000).astype(np.float32).astype(np.float64)
    hi, lo = P.split_bf16(x)
    assert np.array_equal(P.round_bf16(hi), hi) and np.array_equal(P.round_bf16(lo), lo)
    assert np.all(np.abs(lo) <= 2.0 ** -8 * np.abs(x))
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -16 * np.abs(x))
    # a value already in bfloat16 has no low part
    h2, l2 = P.split_bf16(hi)
    assert np.array_equal(h2, hi) and not np.any(l2)


def test_ttm_bf16_elementwise_loops():
    g = np.random.default_rng(7)
    X = g.standard_normal((2, 5, 3)).astype(np.float32)
    A = g.standard_normal((4, 5)).astype(np.float32)  # K x L
    Z = P.ttm_bf16(X, A, 1)
    for a in range(2):
        for k in range(4):
            for b in range(3):
                s = 0.0
                for l in range(5):
                    s += float(P.round_bf16(A[k, l])) * float(P.round_bf16(X[a, l, b]))
                assert abs(Z[a, k, b] - s) <= 1e-14 * (1 + abs(s))


def test_bf16_and_bf16x3_error_levels():
    g = np.random.default_rng(8)
    X = g.standard_normal((6, 64, 50)).astype(np.float32)
    A = g.standard_normal((20, 64)).astype(np.float32)
    exact = O.ttm(X, A, 1)
    nrm = np.linalg.norm(exact)
    e16 = np.linalg.norm(P.ttm_bf16(X, A, 1) - exact) / nrm
    e3 = np.linalg.norm(P.ttm_bf16x3(X, A, 1) - exact) / nrm
    # one rounding of each operand: relative error of order 2^-8
    assert 1e-4 < e16 < 1e-2
    # representation error 2^-16 per operand plus the dropped lo*lo term
    assert 1e-8 < e3 < 1e-4
    # with X already in bfloat16, two products reproduce the three-product form
    Xb = P.round_bf16(X)
    np.testing.assert_allclose(P.ttm_bf16x3(Xb, A, 1, x_is_bf16=True),
                               P.ttm_bf16x3(Xb, A, 1), rtol=0, atol=1e-12)
    # dropping a kept product is detectable at this size
    Xh, Xl = P.split_bf16(X)
    Ah, Al = P.split_bf16(A)
    two = O.ttm(Xh, Ah, 1) + O.ttm(Xh, Al, 1)
    assert np.linalg.norm(two - exact) / nrm > 1e-4
