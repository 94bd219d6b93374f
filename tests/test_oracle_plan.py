"""Pins of the planning oracle: the dynamic program against brute-force
enumeration of trees, closed forms and the counter-example of Sec. 3.3."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import plan as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _size(L):
    s = 1
    for x in L:
        s *= x
    return s


def _random_shape(g, N):
    L = [int(g.choice([2, 3, 5, 8, 20, 50, 100, 400])) for _ in range(N)]
    K = [int(g.integers(1, l + 1)) for l in L]
    return L, K


def test_python_and_c_enumerators_agree():
    g = np.random.default_rng(11)
    for _ in range(20):
        N = int(g.integers(2, 5))
        L, K = _random_shape(g, N)
        py = sorted(c for c, _ in P.brute_force_py(L, K))
        bf = P.brute_force(L, K, k=min(len(py), 256))
        assert bf["min_cost"] == py[0]
        assert bf["min_count"] == py.count(py[0])
        assert [c for c, _ in bf["best"]] == py[:len(bf["best"])]


@pytest.mark.parametrize("N", [2, 3, 4])
def test_dp_equals_brute_force_small(N):
    # Lemma 3.1 + recurrence: the binary-tree DP reaches the optimum over all tries
    g = np.random.default_rng(20 + N)
    for _ in range(60):
        L, K = _random_shape(g, N)
        cost, tree = P.optimal_tree(L, K)
        P.validate(tree, N)
        assert P.tree_cost(L, K, tree) == cost
        bf = P.brute_force(L, K, k=256)
        assert cost == bf["min_cost"]
        if bf["min_count"] <= len(bf["best"]):
            opt = {P.canonical(t) for c, t in bf["best"] if c == cost}
            assert P.canonical(tree) in opt


def test_dp_equals_brute_force_five_modes():
    g = np.random.default_rng(55)
    for _ in range(6):
        L, K = _random_shape(g, 5)
        cost, tree = P.optimal_tree(L, K)
        assert cost == P.brute_force(L, K, k=1)["min_cost"]


def test_closed_form_64cube_rank8():
    # two distinct root children cost 2 K |T|, three depth-2 nodes 3 K h |T|: 19 |T|
    L, K = (64, 64, 64), (8, 8, 8)
    cost, tree = P.optimal_tree(L, K)
    assert cost == 19 * _size(L) == 4_980_736
    assert P.tree_cost(L, K, P.chain_tree(3)) == 27 * _size(L) == 7_077_888
    assert P.canonical(tree) == "T(m0(m1(F2),m2(F1)),m1(m2(F0)))"
    assert P.brute_force(L, K, k=16)["min_count"] == 6


def test_closed_form_200_4_rank20():
    # 2 K (1 + h + h) |T| ... = 2 (20 + 2 + 2*0.2) |T| = 44.8 |T|; naive chain 88.8 |T|
    L, K = (200,) * 4, (20,) * 4
    cost, tree = P.optimal_tree(L, K)
    assert cost * 10 == 448 * _size(L)
    assert P.tree_cost(L, K, P.chain_tree(4)) * 10 == 888 * _size(L)
    assert P.brute_force(L, K, k=16)["min_count"] == 12


def test_remark_forced_reuse_is_not_optimal():
    # Sec. 3.3 Remarks: always reusing when R is non-empty can lose.
    L, K = (100, 50, 400, 3, 2), (80, 25, 40, 1, 1)
    opt, _ = P.optimal_tree(L, K)
    forced, _ = P.optimal_tree(L, K, forced_reuse=True)
    assert opt == P.brute_force(L, K, k=1)["min_cost"] == 597_800_000
    assert forced == 601_620_000 > opt


def test_single_chain_order_closed_form():
    g = np.random.default_rng(77)
    for _ in range(200):
        N = int(g.integers(2, 7))
        L, K = _random_shape(g, N)
        for n in range(N):
            others = [j for j in range(N) if j != n]
            best = min(P.chain_cost(L, K, p) for p in itertools.permutations(others))
            assert P.chain_cost(L, K, P.single_chain_order(L, K, n)) == best
            assert P.optimal_state_cost(L, K, 0, 1 << n) == best


def test_prior_scheme_trees_are_valid():
    for N in range(2, 8):
        P.validate(P.chain_tree(N), N)
        P.validate(P.balanced_tree(N), N)
        L = list(range(3, 3 + N))
        K = [max(1, l // 2) for l in L]
        for key in ("K", "h"):
            P.validate(P.ordered_chain_tree(L, K, key), N)
    # balanced tree for N = 4 (Sec. 3.2): about N log N internal nodes
    assert len(P.tree_nodes(P.balanced_tree(4))) == 8
    assert len(P.tree_nodes(P.chain_tree(4))) == 12


def test_golden_plans():
    with open(os.path.join(GOLDEN, "plans.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        cost, tree = P.optimal_tree(case["L"], case["K"])
        assert cost == case["dp_cost"]
        assert P.canonical(tree) == case["dp_tree"]
