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


# ---------------------------------------------------------------------------
# Literal pins, each derived by hand below (not by the oracle)
# ---------------------------------------------------------------------------
def test_literal_optimal_plans_of_the_workloads():
    """Canonical optimal trees and their multiply-add counts (Sec. 3.1 cost
    K_n |In(u)|) for the 200^4, 80^5 and six-mode workloads.

    80^5, K = 10 (h = 1/8), |T| = 3,276,800,000, tree
    T(m0(m1(m2(m3(F4),m4(F3)),m3(m4(F2)))),m2(m3(m4(m0(F1),m1(F0))))):
      root children m0, m2:               2 * 10 |T|            = 20 |T|
      m1 under m0, m3 under m2:           2 * 10 |T| / 8        = 2.5 |T|
      m2, m3 under m0.m1; m4 under m2.m3: 3 * 10 |T| / 64       = 0.46875 |T|
      m3, m4 under m0.m1.m2; m4 under m0.m1.m3; m0, m1 under m2.m3.m4:
                                          5 * 10 |T| / 512      = 0.09765625 |T|
      total 23.06640625 |T| = 75,584,000,000.
    200^4, K = 20 (h = 1/10): 2 * 20 (1 + 2 h + 2 h^2) |T| = 44.8 |T|
      = 71,680,000,000.
    Six-mode 64x48x40x32x24x16, K = (8,8,6,6,4,4), |T| = 1,509,949,440: the
    string below; its cost node by node (input sizes as products of the
    current dimensions):
      m4: 4 |T| = 6,039,797,760; m5: 4 |T| = 6,039,797,760  (root children)
      under m4 (64x48x40x32x4x16 = 251,658,240): m3 6 * 251,658,240
        = 1,509,949,440 -> 64x48x40x6x4x16 (47,185,920): m1 8 * 47,185,920
        = 377,487,360 -> 64x8x40x6x4x16 (7,864,320): m2 6 * 7,864,320
        = 47,185,920 -> 64x8x6x6x4x16 (1,179,648): m0 8 * 1,179,648
        = 9,437,184 -> F5 and m5 4 * 1,179,648 = 4,718,592 -> F0;
        m5 under m4.m3.m1 (7,864,320): 4 * 7,864,320 = 31,457,280
        -> 64x8x40x6x4x4 (1,966,080): m0 8 * 1,966,080 = 15,728,640 -> F2
      under m5 (64x48x40x32x24x4 = 377,487,360): m2 6 * 377,487,360
        = 2,264,924,160 -> 64x48x6x32x24x4 (56,623,104): m0 8 * 56,623,104
        = 452,984,832 -> 8x48x6x32x24x4 (7,077,888): m3 6 * 7,077,888
        = 42,467,328 -> 8x48x6x6x24x4 (1,327,104): m1 8 * 1,327,104
        = 10,616,832 -> F4 and m4 4 * 1,327,104 = 5,308,416 -> F1;
        m4 under m5.m2.m0 (7,077,888): 4 * 7,077,888 = 28,311,552
        -> 8x48x6x32x4x4 (1,179,648): m1 8 * 1,179,648 = 9,437,184 -> F3
      sum 16,889,610,240."""
    cases = [
        ((200,) * 4, (20,) * 4, "T(m0(m1(m2(F3),m3(F2))),m2(m3(m0(F1),m1(F0))))",
         71_680_000_000),
        ((80,) * 5, (10,) * 5,
         "T(m0(m1(m2(m3(F4),m4(F3)),m3(m4(F2)))),m2(m3(m4(m0(F1),m1(F0)))))",
         75_584_000_000),
        ((64, 48, 40, 32, 24, 16), (8, 8, 6, 6, 4, 4),
         "T(m4(m3(m1(m2(m0(F5),m5(F0)),m5(m0(F2))))),m5(m2(m0(m3(m1(F4),m4(F1)),m4(m1(F3))))))",
         16_889_610_240),
    ]
    six = [6_039_797_760, 6_039_797_760, 1_509_949_440, 377_487_360, 47_185_920, 9_437_184,
           4_718_592, 31_457_280, 15_728_640, 2_264_924_160, 452_984_832, 42_467_328,
           10_616_832, 5_308_416, 28_311_552, 9_437_184]
    assert sum(six) == 16_889_610_240
    assert 3_276_800_000 * 2_306_640_625 == 75_584_000_000 * 10 ** 8
    for L, K, text, macs in cases:
        cost, tree = P.optimal_tree(L, K)
        assert P.canonical(tree) == text
        assert cost == macs
    # the six-mode tree's 16 internal node costs, as listed above
    _, tree6 = P.optimal_tree(*cases[2][:2])
    L6, K6 = cases[2][:2]
    node_costs = sorted(K6[m] * P.card(L6, K6, pm) for _, m, pm in P.tree_nodes(tree6))
    assert node_costs == sorted(six)


def test_ordered_chains_hand_worked():
    """Chain trees of Sec. 3.2 with K-ordering (increasing K_n) and
    h-ordering (increasing h_n = K_n / L_n) on L = (100, 50, 400, 3),
    K = (80, 25, 40, 1), |T| = 6,000,000.

    K-order 3, 1, 2, 0 (K = 1, 25, 40, 80); each leaf's chain skips its mode:
      F0: m3 6e6 (-> 2e6), m1 25*2e6 = 50e6 (-> 1e6), m2 40*1e6 = 40e6:  96e6
      F1: m3 6e6, m2 40*2e6 = 80e6 (-> 2e5), m0 80*2e5 = 16e6:          102e6
      F2: m3 6e6, m1 50e6 (-> 1e6), m0 80*1e6 = 80e6:                   136e6
      F3: m1 25*6e6 = 150e6 (-> 3e6), m2 120e6 (-> 3e5), m0 24e6:       294e6
      total 628,000,000.
    h-order 2, 3, 1, 0 (h = 0.1, 1/3, 0.5, 0.8):
      F0: m2 40*6e6 = 240e6 (-> 6e5), m3 6e5 (-> 2e5), m1 25*2e5 = 5e6: 245.6e6
      F1: m2 240e6, m3 6e5, m0 80*2e5 = 16e6:                           256.6e6
      F2: m3 6e6, m1 50e6, m0 80e6:                                     136e6
      F3: m2 240e6 (-> 6e5), m1 25*6e5 = 15e6 (-> 3e5), m0 24e6:        279e6
      total 917,200,000.
    Ties go to the lower mode: K = (4, 4, 2) orders 2, 0, 1.  Leaf chains,
    K-order: F0 m3.m1.m2, F1 m3.m2.m0, F2 m3.m1.m0, F3 m1.m2.m0; h-order:
    F0 m2.m3.m1, F1 m2.m3.m0, F2 m3.m1.m0, F3 m2.m1.m0."""
    L, K = (100, 50, 400, 3), (80, 25, 40, 1)
    assert P.mode_order(L, K, "K") == [3, 1, 2, 0]
    assert P.mode_order(L, K, "h") == [2, 3, 1, 0]
    assert P.mode_order((8, 9, 10), (4, 4, 2), "K") == [2, 0, 1]
    assert P.mode_order((8, 16, 10), (4, 8, 5), "h") == [0, 1, 2]  # all h = 1/2
    tk_ = P.ordered_chain_tree(L, K, "K")
    th = P.ordered_chain_tree(L, K, "h")
    # one independent chain per leaf, children sorted as strings
    assert P.canonical(tk_) == "T(m1(m2(m0(F3))),m3(m1(m0(F2))),m3(m1(m2(F0))),m3(m2(m0(F1))))"
    assert P.canonical(th) == "T(m2(m1(m0(F3))),m2(m3(m0(F1))),m2(m3(m1(F0))),m3(m1(m0(F2))))"
    assert P.tree_cost(L, K, tk_) == 628_000_000
    assert P.tree_cost(L, K, th) == 917_200_000
    assert P.chain_cost(L, K, [2, 3, 1]) == 245_600_000
    assert P.chain_cost(L, K, [3, 1, 2]) == 96_000_000


def test_balanced_tree_hand_worked():
    """Balanced tree of Sec. 3.2 on modes 0..3: {0,1} | {2,3}, so the root's
    children are the chains m0.m1 (above m2 -> F3 and m3 -> F2) and m2.m3
    (above m0 -> F1 and m1 -> F0).  On L = (100, 50, 400, 3),
    K = (80, 25, 40, 1), |T| = 6e6:
      m0 80*6e6 = 480e6 (-> 4.8e6), m1 25*4.8e6 = 120e6 (-> 2.4e6),
      m2 40*2.4e6 = 96e6, m3 1*2.4e6 = 2.4e6;
      m2 40*6e6 = 240e6 (-> 6e5), m3 6e5 (-> 2e5), m0 80*2e5 = 16e6,
      m1 25*2e5 = 5e6;
      total 960,000,000.
    At 200^4 rank 20 it is the optimal tree itself (44.8 |T|)."""
    t = P.balanced_tree(4)
    assert P.canonical(t) == "T(m0(m1(m2(F3),m3(F2))),m2(m3(m0(F1),m1(F0))))"
    assert P.tree_cost((100, 50, 400, 3), (80, 25, 40, 1), t) == 960_000_000
    assert P.tree_cost((200,) * 4, (20,) * 4, t) == 71_680_000_000
    # five modes: {0,1} | {2,3,4}; the second group splits {2} | {3,4}
    t5 = P.balanced_tree(5)
    assert P.canonical(t5) == ("T(m0(m1(m2(m3(F4),m4(F3)),m3(m4(F2)))),"
                               "m2(m3(m4(m0(F1),m1(F0)))))")
