"""TTM-tree planning oracle -- test infrastructure only.

Trees are nested tuples:
    ("T", children)            the root, labelled with the input tensor
    ("m", n, children)         an internal node: TTM along mode n
    ("F", n)                   a leaf: the new factor matrix of mode n
Modes are 0-based here (the paper numbers them from 1).

Cost model (Sec. 3.1, "Computational Load"): an internal node with mode n
costs K_n * |In(u)| multiply-adds and outputs |Out(u)| = (K_n / L_n) |In(u)|.
The root's output is T itself.  Costs are exact Python integers.

Optimal tree (Sec. 3.3): dynamic program over triples (P, Q, R) -- modes
already multiplied, leaves still to build below this node, modes that may be
reused.  Readings of the garbled / silent points (listed in the design notes):
  * a split of Q into Q1, Q2 hands each half the other half as extra reusable
    modes: (P, Q1, R u Q2) and (P, Q2, R u Q1).  With this reading R is fixed by
    P and Q (R = [N] minus P minus Q) and every state is a pair (P, Q);
  * ties: reuse candidates in ascending mode first, then splits Q1 (containing
    the lowest mode of Q, Q1 != Q) in ascending bitmask order; the first strict
    minimum is kept;
  * canonical text: leaf "F<n>", node "m<n>(...)", root "T(...)", children
    sorted as strings and joined by ",".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction
from functools import lru_cache

_HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Sec. 3.1: tree cost
# --------------------------------------------------------------------------
def card(L, K, P_mask: int) -> int:
    """|T[P]|: cardinality of T after multiplying along the modes in P."""
    c = 1
    for j in range(len(L)):
        c *= int(K[j]) if (P_mask >> j) & 1 else int(L[j])
    return c


def tree_cost(L, K, tree) -> int:
    """Sum over internal nodes of K_n * |In(u)| (top-down)."""
    total = 0

    def visit(node, size_in):
        nonlocal total
        if node[0] == "F":
            return
        n, kids = node[1], node[2]
        total += int(K[n]) * size_in
        size_out = size_in // int(L[n]) * int(K[n])
        for c in kids:
            visit(c, size_out)

    size_T = 1
    for x in L:
        size_T *= int(x)
    for c in tree[1]:
        visit(c, size_T)
    return total


def tree_nodes(tree):
    """Internal nodes as (depth, mode, P_mask_of_input) in depth-first order."""
    out = []

    def visit(node, depth, P):
        if node[0] == "F":
            return
        out.append((depth, node[1], P))
        for c in node[2]:
            visit(c, depth + 1, P | (1 << node[1]))

    for c in tree[1]:
        visit(c, 0, 0)
    return out


def canonical(tree) -> str:
    """Canonical text form (children sorted as strings)."""
    if tree[0] == "F":
        return f"F{tree[1]}"
    if tree[0] == "m":
        return f"m{tree[1]}(" + ",".join(sorted(canonical(c) for c in tree[2])) + ")"
    return "T(" + ",".join(sorted(canonical(c) for c in tree[1])) + ")"


def validate(tree, N: int) -> None:
    """Check the TTM-tree properties of Sec. 3.1: N unique leaves, each path
    holding every other mode exactly once.  Raises ValueError otherwise."""
    if tree[0] != "T":
        raise ValueError("root must be T")
    seen = set()

    def visit(node, path):
        if node[0] == "F":
            n = node[1]
            if n in seen:
                raise ValueError(f"leaf F{n} appears twice")
            seen.add(n)
            if sorted(path) != [j for j in range(N) if j != n]:
                raise ValueError(f"path to F{n} is {path}")
            return
        if node[0] != "m" or not node[2]:
            raise ValueError("internal node without children")
        for c in node[2]:
            visit(c, path + [node[1]])

    for c in tree[1]:
        visit(c, [])
    if seen != set(range(N)):
        raise ValueError(f"leaves {sorted(seen)} != all modes")


# --------------------------------------------------------------------------
# Sec. 3.3: the optimal-tree dynamic program
# --------------------------------------------------------------------------
def _bits(mask: int):
    j = 0
    while mask:
        if mask & 1:
            yield j
        mask >>= 1
        j += 1


def optimal_tree(L, K, forced_reuse: bool = False):
    """Minimum-cost TTM-tree by the recurrence of Sec. 3.3.

    cost(P, Q) = min( min_{n in R} K_n |T[P]| + cost(P + {n}, Q),            (reuse)
                      min_{Q1 + Q2 = Q} cost(P, Q1) + cost(P, Q2) )          (split)
    with R = [N] - P - Q; base case |Q| = 1, R empty: cost 0.
    forced_reuse=True forbids splitting while R is non-empty (the strategy the
    Remarks of Sec. 3.3 show to be sub-optimal).
    Returns (cost, tree).
    """
    N = len(L)
    full = (1 << N) - 1

    @lru_cache(maxsize=None)
    def solve(P: int, Q: int):
        R = full & ~(P | Q)
        if R == 0 and Q & (Q - 1) == 0:
            return 0, (("F", Q.bit_length() - 1),)
        best = None
        size = card(L, K, P)
        for n in _bits(R):
            sub_cost, sub = solve(P | (1 << n), Q)
            c = int(K[n]) * size + sub_cost
            if best is None or c < best[0]:
                best = (c, (("m", n, sub),))
        if not (forced_reuse and R != 0):
            low = Q & -Q
            Q1 = 0
            while True:
                Q1 = (Q1 - Q) & Q          # next submask of Q, ascending
                if Q1 == Q or Q1 == 0:
                    break
                if not Q1 & low:
                    continue
                c1, f1 = solve(P, Q1)
                c2, f2 = solve(P, Q ^ Q1)
                if best is None or c1 + c2 < best[0]:
                    best = (c1 + c2, f1 + f2)
        return best

    cost, forest = solve(0, full)
    return cost, ("T", forest)


def optimal_state_cost(L, K, P: int, Q: int) -> int:
    """cost(P, Q) of the dynamic program for one sub-problem."""
    N = len(L)
    full = (1 << N) - 1
    # solve on a fresh table restricted to this state
    memo = {}

    def solve(P, Q):
        key = (P, Q)
        if key in memo:
            return memo[key]
        R = full & ~(P | Q)
        if R == 0 and Q & (Q - 1) == 0:
            memo[key] = 0
            return 0
        best = None
        size = card(L, K, P)
        for n in _bits(R):
            c = int(K[n]) * size + solve(P | (1 << n), Q)
            best = c if best is None or c < best else best
        low = Q & -Q
        Q1 = 0
        while True:
            Q1 = (Q1 - Q) & Q
            if Q1 == Q or Q1 == 0:
                break
            if Q1 & low:
                c = solve(P, Q1) + solve(P, Q ^ Q1)
                best = c if best is None or c < best else best
        memo[key] = best
        return best

    return solve(P, Q)


# --------------------------------------------------------------------------
# Sec. 3.2: prior schemes
# --------------------------------------------------------------------------
def _chain(modes, below):
    node = below
    for m in reversed(list(modes)):
        node = (("m", m, node),)
    return node


def chain_tree(N: int, orders=None):
    """Chain tree: N independent chains, leaf n's chain follows orders[n]
    (default ascending modes, the naive scheme)."""
    kids = []
    for n in range(N):
        order = orders[n] if orders is not None else [j for j in range(N) if j != n]
        kids.extend(_chain(order, (("F", n),)))
    return ("T", tuple(kids))


def mode_order(L, K, key: str):
    """K-ordering (increasing K_n) or h-ordering (increasing K_n / L_n); ties by mode."""
    N = len(L)
    if key == "K":
        return sorted(range(N), key=lambda j: (int(K[j]), j))
    if key == "h":
        return sorted(range(N), key=lambda j: (Fraction(int(K[j]), int(L[j])), j))
    if key == "naive":
        return list(range(N))
    raise ValueError(key)


def ordered_chain_tree(L, K, key: str):
    order = mode_order(L, K, key)
    N = len(L)
    return chain_tree(N, [[j for j in order if j != n] for n in range(N)])


def balanced_tree(N: int, order=None):
    """Divide-and-conquer tree (Sec. 3.2, balanced trees): split the modes into
    the first floor(|S|/2) and the rest; a chain of the first group leads to the
    recursive tree of the second group, and vice versa."""
    order = list(range(N)) if order is None else list(order)

    def build(S):
        if len(S) == 1:
            return (("F", S[0]),)
        m = len(S) // 2
        S1, S2 = S[:m], S[m:]
        return _chain(S1, build(S2)) + _chain(S2, build(S1))

    return ("T", build(order))


def single_chain_order(L, K, n: int):
    """Cheapest order for one isolated chain (leaf n): ascending K_j / (1 - h_j),
    i.e. K_j L_j / (L_j - K_j), with h_j = 1 modes last.  (Exchange argument on
    two adjacent TTMs of the chain.)"""
    def key(j):
        if int(K[j]) == int(L[j]):
            return (1, Fraction(0), j)
        return (0, Fraction(int(K[j]) * int(L[j]), int(L[j]) - int(K[j])), j)
    return sorted((j for j in range(len(L)) if j != n), key=key)


def chain_cost(L, K, order) -> int:
    """Cost of one chain of TTMs over T in the given mode order."""
    size = 1
    for x in L:
        size *= int(x)
    total = 0
    for j in order:
        total += int(K[j]) * size
        size = size // int(L[j]) * int(K[j])
    return total


# --------------------------------------------------------------------------
# Brute force over tries (plain C, built by build_brute())
# --------------------------------------------------------------------------
_LIB = None


def build_brute() -> str:
    """Compile brute_plan.c into a shared object next to it; return its path."""
    src = os.path.join(_HERE, "brute_plan.c")
    out = os.path.join(_HERE, "libbrute_plan.so")
    subprocess.run(["gcc", "-O2", "-shared", "-fPIC", "-o", out, src], check=True)
    return out


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libbrute_plan.so")
        src = os.path.join(_HERE, "brute_plan.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            build_brute()
        lib = ctypes.CDLL(path)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.brute_plan.argtypes = [ctypes.c_int, u64p, u64p, ctypes.c_int, u64p, u64p,
                                   u64p, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_int)]
        lib.brute_plan.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def tree_from_paths(paths) -> tuple:
    """Merge the N root-to-leaf mode sequences into a trie-shaped tree."""
    N = len(paths)

    def build(prefix_paths, depth):
        # prefix_paths: list of (leaf, path); group by the mode at this depth
        groups = {}
        leaves = []
        for leaf, path in prefix_paths:
            if depth == len(path):
                leaves.append(("F", leaf))
            else:
                groups.setdefault(path[depth], []).append((leaf, path))
        kids = [("m", m, build(g, depth + 1)) for m, g in sorted(groups.items())]
        return tuple(leaves) + tuple(kids)

    return ("T", build([(n, list(paths[n])) for n in range(N)], 0))


def brute_force(L, K, k: int = 16):
    """Enumerate every trie-shaped TTM-tree (N <= 5 in practice).

    Returns dict(min_cost, min_count, best=[(cost, tree), ...] for the k
    cheapest tries, cost ascending).
    """
    N = len(L)
    lib = _lib()
    Lc = (ctypes.c_uint64 * N)(*[int(x) for x in L])
    Kc = (ctypes.c_uint64 * N)(*[int(x) for x in K])
    mc = ctypes.c_uint64()
    cnt = ctypes.c_uint64()
    costs = (ctypes.c_uint64 * max(k, 1))()
    paths = (ctypes.c_int * (max(k, 1) * N * max(N - 1, 1)))()
    nout = ctypes.c_int()
    rc = lib.brute_plan(N, Lc, Kc, k, ctypes.byref(mc), ctypes.byref(cnt), costs, paths,
                        ctypes.byref(nout))
    if rc != 0:
        raise ValueError("brute_plan rejected its arguments")
    best = []
    for i in range(nout.value):
        pl = [[paths[(i * N + n) * (N - 1) + s] for s in range(N - 1)] for n in range(N)]
        best.append((int(costs[i]), tree_from_paths(pl)))
    return dict(min_cost=int(mc.value), min_count=int(cnt.value), best=best)


def brute_force_py(L, K):
    """Pure-Python enumeration of all tries (N <= 4): list of (cost, canonical)."""
    import itertools
    N = len(L)
    perms = [list(itertools.permutations([j for j in range(N) if j != n])) for n in range(N)]
    out = []
    for combo in itertools.product(*perms):
        t = tree_from_paths(combo)
        out.append((tree_cost(L, K, t), canonical(t)))
    return out
