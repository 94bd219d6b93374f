"""Helpers for the GPU tests: device handles and element-wise error bounds.

Element-wise parity.  Every result of a TTM (or a chain of TTMs, or a Gram
product) is a sum of products, and the forward error of a floating-point sum of
n products is bounded element by element by gamma_n times the same sum taken
over the absolute values of its terms:

    |fl(sum_l x_l f_l) - sum_l x_l f_l|  <=  n u / (1 - n u) * sum_l |x_l| |f_l|

(u = unit roundoff of the accumulation), whatever the summation order.  So
each GPU result is compared with the FP64 oracle entry by entry against the
oracle's contraction of |X| and |F| ("magnitude bound"), never through a norm
over the whole array, and a wrong term, index or sign anywhere -- in a ragged
tail included -- shows up in the element it touches.  Operand rounding of the
reduced-precision modes adds a relative term per product:

* fp64: (L + 2) 2^-53
* fp32: (L + 2) 2^-24; FP32 compute on BF16 input runs three exact BF16
  products per term (the factor split into three bfloat16 parts), so
  (3 L + 2) 2^-24
* bf16 (both operands rounded to 8 significant bits, 2^-8 each; products
  exact in FP32): 2^-7 + 2^-16 + (L + 2) 2^-24
* bf16x3 (operand = hi + lo within 2^-16 relative, the lo*lo product
  dropped): 4 * 2^-16 + (3 L + 2) 2^-24

A chain of TTMs adds the bounds of its steps (first order); the magnitude
bound of the chain is the chain over |T| and |F|, which does not depend on
the order of the steps.
"""
import numpy as np

from oracle import hooi as O

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def rel_err(a, b):
    """Normwise relative difference (reported beside the element-wise checks)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm((a - b).reshape(-1))
    n = np.linalg.norm(b.reshape(-1))
    return d / n if n > 0 else d


def ttm_tol(L, compute, bf16_input=False):
    """Per-element bound of one TTM with reduction length L, relative to the
    magnitude bound (see the module docstring)."""
    L = int(L)
    if compute == "fp64":
        return (L + 2) * U64
    if compute == "fp32":
        return ((3 * L + 2) if bf16_input else (L + 2)) * U32
    if compute == "bf16":
        return 2.0 ** -7 + 2.0 ** -16 + (L + 2) * U32
    if compute == "bf16x3":
        return 4 * 2.0 ** -16 + (3 * L + 2) * U32
    raise ValueError(compute)


def chain_tol(Ls, compute, bf16_input=False):
    """First-order bound of a chain of TTMs with reduction lengths Ls."""
    return 1.01 * sum(ttm_tol(L, compute, bf16_input) for L in Ls)


def assert_elementwise(got, ref, bound, tol, what=""):
    """|got - ref| <= tol * bound for every element (bound: magnitude bound,
    an array of ref's shape or a scalar); reports the worst element."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    bound = np.broadcast_to(np.asarray(bound, dtype=np.float64), ref.shape)
    diff = np.abs(got - ref)
    lim = tol * bound
    bad = diff > lim
    if bad.any():
        ratio = np.where(lim > 0, diff / np.where(lim > 0, lim, 1.0), np.inf)
        i = np.unravel_index(int(np.argmax(ratio)), ref.shape)
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {ref.size} elements outside tol {tol:.3e}; "
            f"worst at {i}: got {got[i]!r} ref {ref[i]!r} |diff| {diff[i]:.3e} "
            f"bound {bound[i]:.3e} (normwise rel {rel_err(got, ref):.3e})")
    return float(np.max(diff / np.where(bound > 0, bound, 1.0))) if ref.size else 0.0


def abs_ttm(X, F_T, n):
    """Magnitude bound of a TTM: the oracle's TTM of |X| and |F^T|."""
    return O.ttm(np.abs(X), np.abs(F_T), n)


def abs_chain(T, F, n):
    """Magnitude bound of the naive chain for leaf n: the chain over |T|, |F|."""
    return O.chain_except(np.abs(T), [np.abs(f) for f in F], n)


def abs_gram(Yabs, n):
    """Magnitude bound of a Gram product: the Gram of |Y_(n)|."""
    return O.gram(np.abs(Yabs), n)


def abs_leaf_entries(T, F, n, index_list):
    """Magnitude bounds of sampled leaf entries: the oracle's entry-by-entry
    contraction applied to |T| (one mode-n slice at a time) and |F|."""
    Fa = [np.abs(np.asarray(f, dtype=np.float64)) for f in F]
    out = np.empty(len(index_list), dtype=np.float64)
    for e, idx in enumerate(index_list):
        sl = np.abs(np.take(T, int(idx[n]), axis=n).astype(np.float64))
        sl = np.expand_dims(sl, n)
        j = list(idx)
        j[n] = 0
        out[e] = O.leaf_entries(sl, Fa, n, [tuple(j)])[0]
    return out


def subspace_dist(F1, F2):
    """||F1 F1^T - F2 F2^T||_2 (basis-free comparison of column spaces)."""
    return float(np.linalg.norm(F1 @ F1.T - F2 @ F2.T, 2))


def to_dev(x, dtype=None):
    torch, dev = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)
