"""Reduced-precision TTM models -- test infrastructure only.

The paper computes in double precision; the BF16 and split-BF16 compute modes
are additions of this implementation (its precision modes).  This module
states, in float64, exactly what those modes compute for one TTM node
(Sec. 2.1), so a GPU node can be compared element by element:

* round_bf16(x): the nearest bfloat16 value of x (8 significant bits, ties to
  even), for x in the normal range of float32;
* split_bf16(x): hi = round_bf16(x), lo = round_bf16(x - hi); x - (hi + lo) is
  at most 2^-16 |x|;
* ttm_bf16(X, A, n): TTM of the rounded operands (every product of two 8-bit
  significands is exact; the sum is exact up to float64 rounding);
* ttm_bf16x3(X, A, n): hi*hi + hi*lo + lo*hi with the lo*lo term dropped.

The rounding is written from its definition (significand scaled to 8 bits,
rounded half to even), not from a bit trick, so that it can be checked
against a library cast independently.
"""
from __future__ import annotations

import numpy as np

from .hooi import ttm

BF16_BITS = 8  # significant bits of bfloat16 (7 stored + the implicit one)


def round_bf16(x) -> np.ndarray:
    """Nearest bfloat16 value of every element (ties to even), as float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)  # x = m * 2^e with 0.5 <= |m| < 1 (m = 0 for x = 0)
    r = np.rint(m * 2.0 ** BF16_BITS)  # rint rounds half to even
    return np.ldexp(r, e - BF16_BITS)


def split_bf16(x):
    """(hi, lo) with hi = round_bf16(x), lo = round_bf16(x - hi)."""
    x = np.asarray(x, dtype=np.float64)
    hi = round_bf16(x)
    return hi, round_bf16(x - hi)


def ttm_bf16(X: np.ndarray, A: np.ndarray, n: int) -> np.ndarray:
    """TTM (Sec. 2.1) of X and the K x L matrix A, both rounded to bfloat16."""
    return ttm(round_bf16(X), round_bf16(A), n)


def ttm_bf16x3(X: np.ndarray, A: np.ndarray, n: int, x_is_bf16: bool = False) -> np.ndarray:
    """Split-BF16 TTM: Xh Ah + Xl Ah + Xh Al (the Xl Al term dropped).

    x_is_bf16: X already holds bfloat16 values, so its low part is zero and
    two products remain."""
    Xh, Xl = split_bf16(X)
    Ah, Al = split_bf16(A)
    out = ttm(Xh, Ah, n) + ttm(Xh, Al, n)
    if not x_is_bf16:
        out = out + ttm(Xl, Ah, n)
    return out
