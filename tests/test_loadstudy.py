"""Machine-independent load study (Sec. 6.1 benchmark space, Sec. 6.2 "TTM
computational load") through the library's planner, pinned against the
oracle's planner and the brute-force enumerator of trees.

Host-only: the planner half of the C ABI runs without a GPU."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import plan as P

tk = pytest.importorskip("paper_1707_05594_amd")
from paper_1707_05594_amd import loadstudy as S  # noqa: E402


def _oracle_loads(L, K):
    return {"dp": P.optimal_tree(L, K)[0],
            "chain_k": P.tree_cost(L, K, P.ordered_chain_tree(L, K, "K")),
            "chain_h": P.tree_cost(L, K, P.ordered_chain_tree(L, K, "h")),
            "balanced": P.tree_cost(L, K, P.balanced_tree(len(L)))}


def test_benchmark_space_recipe():
    """K_n = L_n / ratio over {20, 50, 100, 400} x {1.25, 2, 5, 10}, every
    K_n an integer no larger than L_n; |T| <= 8e9."""
    pr = S.pairs()
    assert len(pr) == 16
    assert (400, 320) in pr and (20, 2) in pr and (50, 40) in pr and (100, 10) in pr
    for L, K in pr:
        assert 1 <= K <= L and Fraction(L, K) in S.RATIOS
    for L, K, ok in S.shapes(5):
        assert np.prod(L, dtype=np.int64) <= 8 * 10 ** 9
        assert list(L) == sorted(L)


@pytest.mark.parametrize("shape", [S.PAPER_MIN_GAIN, S.PAPER_MAX_GAIN])
def test_paper_example_tensors(shape):
    """The two tensors Sec. 6.2 names (smallest and largest overall gain):
    every load from the library's planner equals the oracle's, and the
    optimum equals the brute-force minimum over all tries."""
    L, K = shape
    got = S.loads(L, K)
    want = _oracle_loads(L, K)
    assert got == want
    assert got["dp"] == P.brute_force(L, K, k=1)["min_cost"]
    assert all(got[k] > got["dp"] for k in S.PRIOR)  # the optimum beats every prior scheme here
    print(f"{L} -> {K}: best prior / optimal {S.ratio(got):.4f}")


def test_sampled_shapes_match_oracle():
    """A seeded sample of the 5-D and 6-D spaces (ordered tuples): the four
    loads of every sampled shape equal the oracle's."""
    g = np.random.default_rng(61)
    choices = S.pairs()
    done = 0
    while done < 120:
        N = 5 if done < 80 else 6
        combo = [choices[int(i)] for i in g.integers(0, len(choices), size=N)]
        L = tuple(c[0] for c in combo)
        K = tuple(c[1] for c in combo)
        if np.prod(L, dtype=np.int64) > 8e9 or not S.feasible(K):
            continue
        assert S.loads(L, K) == _oracle_loads(L, K), (L, K)
        done += 1


def test_study_extremes_over_multisets():
    """The largest best-prior / optimal load ratios of the multiset spaces,
    recomputed with the oracle: 5-D (20, 50, 100, 100, 400) -> (10, 10, 80,
    10, 40) and 6-D 20^6 -> (10, 2, 2, 2, 2, 2); and each is the study's
    maximum."""
    cases = {5: (((20, 50, 100, 100, 400), (10, 10, 80, 10, 40)), 2.5124),
             6: (((20,) * 6, (10, 2, 2, 2, 2, 2)), 2.9802)}
    for N, ((L, K), r) in cases.items():
        ld = _oracle_loads(L, K)
        ro = min(ld[k] for k in S.PRIOR) / ld["dp"]
        assert abs(ro - r) < 5e-5
        rows, _ = S.study(N)
        s = S.summarise(rows)
        assert s["argmax"] == (L, K)
        assert abs(s["max_ratio"] - ro) < 1e-12
