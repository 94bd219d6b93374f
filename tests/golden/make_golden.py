"""Writes tests/golden/plans.json from the oracle alone (oracle.plan).

Each case: mode lengths L, core lengths K, the dynamic program's optimal cost
(multiply-adds, Sec. 3.1 cost model) and canonical tree (Sec. 3.3 recurrence
with the tie rule stated in oracle/plan.py), the naive chain and balanced tree
costs (Sec. 3.2), and -- where N <= 5 -- the brute-force minimum, its tie
count and the 8 cheapest trie costs.
Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import plan as P  # noqa: E402

CASES = [
    ("64x64x64 ranks 8", (64, 64, 64), (8, 8, 8)),
    ("200^4 ranks 20", (200,) * 4, (20,) * 4),
    ("80^5 ranks 10", (80,) * 5, (10,) * 5),
    ("64x48x40x32x24x16 ranks 8,8,6,6,4,4", (64, 48, 40, 32, 24, 16), (8, 8, 6, 6, 4, 4)),
    ("Remark counter-example", (100, 50, 400, 3, 2), (80, 25, 40, 1, 1)),
    ("min-gain benchmark tensor", (400, 400, 20, 20, 20), (320, 40, 10, 10, 10)),
    ("max-gain benchmark tensor", (400, 100, 100, 50, 20), (80, 80, 10, 40, 10)),
    ("HCCI shape", (672, 672, 627, 16), (279, 279, 153, 14)),
    ("TJLR shape", (460, 700, 360, 16, 4), (306, 232, 239, 16, 4)),
    ("SP shape", (500, 500, 500, 11, 10), (81, 129, 127, 7, 6)),
]


def main():
    out = []
    for name, L, K in CASES:
        cost, tree = P.optimal_tree(L, K)
        case = dict(name=name, L=list(L), K=list(K), dp_cost=cost, dp_tree=P.canonical(tree),
                    naive_chain_cost=P.tree_cost(L, K, P.chain_tree(len(L))),
                    balanced_cost=P.tree_cost(L, K, P.balanced_tree(len(L))))
        if len(L) <= 5:
            bf = P.brute_force(L, K, k=8)
            case.update(brute_min=bf["min_cost"], brute_ties=bf["min_count"],
                        brute_top8=[c for c, _ in bf["best"]])
        out.append(case)
    with open(os.path.join(HERE, "plans.json"), "w") as f:
        json.dump(dict(generator="tests/golden/make_golden.py (oracle.plan only)",
                       cases=out), f, indent=1)


if __name__ == "__main__":
    main()
