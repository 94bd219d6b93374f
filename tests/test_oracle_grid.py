"""Pins of the processor-grid oracle (Sec. 4): the count of grids against the
paper's table and direct enumeration, hand-worked static volumes, and the
dynamic-gridding recurrence against brute force over every scheme."""
import numpy as np
import pytest

from oracle import grid as Gr
from oracle import plan as P


def test_psi_matches_the_papers_table_and_enumeration():
    """Sec. 4.2 "Number of grids": psi(P, N) = prod_i C(e_i + N - 1, N - 1).
    The table's entry for P = 2^5, N = 7 reads 562; the formula gives
    C(11, 6) = 462 (a typo: every other entry matches, the two large ones as
    rounded, 880K for 888,030 and 230K for 230,230)."""
    table = {
        2 ** 5: [126, 252, 562, 792, 1287, 2002],
        2 ** 10: [1001, 3003, 8008, 19448, 43758, 92378],
    }
    for Pn, row in table.items():
        for N, printed in zip(range(5, 11), row):
            got = Gr.psi(Pn, N)
            if (Pn, N) == (2 ** 5, 7):
                assert printed == 562 and got == 462
            else:
                assert got == printed
    big = [10626, 53130, 230_230, 888_030, 3_108_105, 10_015_005]
    for N, v in zip(range(5, 11), big):
        assert Gr.psi(2 ** 20, N) == v
    # rounded as printed: 230K, 880K, 3.1M, 10M
    assert round(big[2], -4) == 230_000 and big[3] // 10 ** 4 == 88
    for Pn in (1, 6, 12, 36, 64, 90):
        for N in (1, 2, 3, 4):
            gs = Gr.grids(Pn, N)
            assert len(gs) == len(set(gs)) == Gr.psi(Pn, N)
            assert all(int(np.prod(g)) == Pn for g in gs)


def test_static_volumes_hand_worked():
    """64^3, K = 8, optimal tree T(m0(m1(F2),m2(F1)),m1(m2(F0))): outputs
    m0 32768, m0.m1 4096, m0.m2 4096, m1 32768, m1.m2 4096.  With P = 8:
      <1,1,8>: mode-2 nodes 7 * (4096 + 4096)             = 57344
      <2,1,4>: 1 * 32768 + 3 * 8192                        = 57344 (tie)
      <2,2,2>: 32768 + 4096 + 4096 + 32768 + 4096          = 77824
      <8,1,1>: 7 * 32768                                   = 229376
      <1,2,4>: 36864 + 3 * 8192                            = 61440
    The optimum is 57344, first reached at <1,1,8>."""
    L, K = (64, 64, 64), (8, 8, 8)
    _, tree = P.optimal_tree(L, K)
    assert P.canonical(tree) == "T(m0(m1(F2),m2(F1)),m1(m2(F0)))"
    want = {(1, 1, 8): 57344, (2, 1, 4): 57344, (2, 2, 2): 77824, (8, 1, 1): 229376,
            (1, 2, 4): 61440}
    for g, v in want.items():
        assert Gr.static_volume(L, K, tree, g) == v
    assert Gr.optimal_static(L, K, tree, 8) == (57344, (1, 1, 8))
    # every static scheme is a dynamic one that never regrids
    assert Gr.dynamic_volume(L, K, tree, (1, 1, 8), [(1, 1, 8)] * 5) == 57344


def test_validity_excludes_grids_beyond_the_core():
    """Valid grids keep q_n <= K_n; with K = (2, 8, 8) and P = 8 the grid
    <8,1,1> is excluded, and with K = (1, 1, 1) no grid of P = 2 is valid."""
    L, K = (64, 64, 64), (2, 8, 8)
    _, tree = P.optimal_tree(L, K)
    v, g = Gr.optimal_static(L, K, tree, 8)
    assert g[0] <= 2
    assert Gr.optimal_static((4, 4, 4), (1, 1, 1), P.chain_tree(3), 2) is None


CASES = [  # (modes, tree kind, P): at most ~5e4 schemes for the brute force
    (3, "dp", 4), (3, "dp", 4), (3, "balanced", 4), (3, "chain", 2), (3, "dp", 3), (4, "dp", 2),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_dynamic_recurrence_equals_brute_force(case):
    """Sec. 4.4 recurrence over (node, parent grid) pairs = the minimum over
    every root grid and every assignment of valid grids to the nodes; never
    above the optimal static grid."""
    N, kind, Pn = CASES[case]
    g = np.random.default_rng(300 + case)
    L = [int(x) for x in g.choice([4, 6, 8, 12], size=N)]
    K = [int(g.integers(2, l + 1)) for l in L]
    if kind == "dp":
        _, tree = P.optimal_tree(L, K)
    elif kind == "chain":
        tree = P.chain_tree(N)
    else:
        tree = P.balanced_tree(N)
    res = Gr.optimal_dynamic(L, K, tree, Pn)
    st = Gr.optimal_static(L, K, tree, Pn)
    if st is None:
        assert res is None
        return
    vol, g0, pi = res
    assert vol == Gr.dynamic_volume(L, K, tree, g0, pi)
    assert vol == Gr.brute_dynamic(L, K, tree, Pn)
    assert vol <= st[0]


# ---------------------------------------------------------------------------
# the library's planner (host-only half of the C ABI) against the oracle
# ---------------------------------------------------------------------------
def _abi_volume(plan, root, per):
    """Volume of the library's scheme, recomputed from its node list by the
    definition: TTM volume per internal node plus |In(u)| per regrid."""
    nodes = plan.nodes()
    vol = 0
    for u, nd in enumerate(nodes):
        if nd["is_leaf"]:
            continue
        pg = root if nd["parent"] < 0 else per[nd["parent"]]
        vol += (per[u][nd["mode"]] - 1) * nd["out_card"]
        if per[u] != pg:
            vol += nd["in_card"]
    return vol


def test_library_grid_count():
    tk = pytest.importorskip("paper_1707_05594_amd")
    for Pn in (1, 2, 6, 32, 64, 90, 1024, 2 ** 20, 3 * 5 * 7 * 11):
        for N in (1, 2, 3, 5, 7, 10):
            assert tk.grid_count(Pn, N) == Gr.psi(Pn, N)


@pytest.mark.parametrize("seed", range(8))
def test_library_grids_match_oracle(seed):
    """Static and dynamic schemes of the library's planner: the same optimal
    volumes as the oracle's exhaustive search and recurrence, the same static
    grid and layout of T (identical tie rule), and node grids whose volume,
    recomputed from the definition, is the reported optimum."""
    tk = pytest.importorskip("paper_1707_05594_amd")
    g = np.random.default_rng(900 + seed)
    N = int(g.integers(3, 6))
    L = [int(x) for x in g.choice([8, 12, 16, 30, 64], size=N)]
    K = [int(g.integers(1, l + 1)) for l in L]
    for _ in range(4):
        for n in range(N):
            K[n] = min(K[n], int(np.prod([K[m] for m in range(N) if m != n])))
    Pn = int(g.choice([4, 8, 12, 16, 32, 64]))
    kind = ["dp", "chain_k", "balanced"][seed % 3]
    plan = tk.ttm_tree_plan(L, K, kind)
    tree = {"dp": lambda: P.optimal_tree(L, K)[1],
            "chain_k": lambda: P.ordered_chain_tree(L, K, "K"),
            "balanced": lambda: P.balanced_tree(N)}[kind]()
    assert P.canonical(tree) == plan.string()
    st = Gr.optimal_static(L, K, tree, Pn)
    if st is None:
        with pytest.raises(tk.TuckerError) as e:
            plan.grids(Pn, "static")
        assert e.value.code == tk.TK_EUNSUPPORTED
        return
    vol, root, per = plan.grids(Pn, "static")
    assert (vol, root) == st
    assert all(p == root for p in per)
    dv, g0, _ = Gr.optimal_dynamic(L, K, tree, Pn)
    vol, root, per = plan.grids(Pn, "dynamic")
    assert vol == dv and root == g0
    assert _abi_volume(plan, root, per) == vol
    assert vol <= st[0]
