"""The allocation-free Gram entry point (tk_gram_noalloc) against tk_gram and
the FP64 oracle, through the C ABI, on two calls in a row (the second with a
smaller input, so the shared scratch area holds the first call's partials).

Bar: element-wise within twice the FP64 bound of a sum of C exact products,
2 (C + 2) 2^-53 of the Gram of |Y| (both entry points round in FP64, in
different chunk orders when the scratch area forces longer chunks)."""
import numpy as np
import pytest

import synth
from oracle import hooi as O
from tests.gpu_util import abs_gram, assert_elementwise, to_dev, torch_dev

pytestmark = pytest.mark.gpu
tk = pytest.importorskip("paper_1707_05594_amd")

CALLS = [
    # (A, L, B, dtype): 1000 rows need 136 tile pairs, so the scratch area
    # takes 7 chunks where tk_gram uses 24; then a small ragged BF16 input
    ((3, 1000, 1000, "f32")),
    ((5, 70, 33, "bf16")),
]


def test_gram_noalloc_matches_gram_twice():
    torch, dev = torch_dev()
    for A, L, B, dtype in CALLS:
        print(f"gram_noalloc A={A} L={L} B={B} {dtype}", flush=True)
        g = np.random.default_rng(A + L + B)
        Y = g.standard_normal((A, L, B)).astype(np.float32)
        if dtype == "bf16":
            bits = synth.round_to_bf16_bits(Y)
            Yd = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).to(dev)
            Y64 = O.as_f64(bits, "bf16")
        else:
            Yd = to_dev(Y)
            Y64 = Y.astype(np.float64)
        S_ref = torch.empty((L, L), dtype=torch.float64, device=dev)
        S_na = torch.full((L, L), float("nan"), dtype=torch.float64, device=dev)
        tk.gram(Yd, A, L, B, S_ref)
        tk.gram_noalloc(Yd, A, L, B, S_na)
        torch.cuda.synchronize()
        got, ref = S_na.cpu().numpy(), S_ref.cpu().numpy()
        mag = abs_gram(Y64, 1)
        tol = 2 * (A * B + 2) * 2.0 ** -53
        assert_elementwise(got, ref, mag, tol, "noalloc vs tk_gram")
        assert_elementwise(got, O.gram(Y64, 1), mag, tol, "noalloc vs oracle")
        np.testing.assert_array_equal(got, got.T)
        # deterministic: a repeat gives the same bits
        S2 = torch.empty_like(S_na)
        tk.gram_noalloc(Yd, A, L, B, S2)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(S2.cpu().numpy(), got)


def test_gram_noalloc_rejects_oversize():
    torch, dev = torch_dev()
    Y = torch.zeros((1, 1100, 4), dtype=torch.float32, device=dev)
    S = torch.zeros((1100, 1100), dtype=torch.float64, device=dev)
    with pytest.raises(tk.TuckerError) as e:
        tk.gram_noalloc(Y, 1, 1100, 4, S)
    assert e.value.code == tk.TK_EUNSUPPORTED
