"""Processor-grid planning oracle (Sec. 4) -- test infrastructure only.

Distributed setup (Sec. 4.1): P processors form an N-dimensional grid
g = <q_1, ..., q_N> with prod q_n = P; every tensor of the tree is cut into P
blocks by it.  The TTM at a node u along mode n then costs a reduce-scatter
of (q_n - 1) |Out(u)| words.  Only valid grids are used: q_n <= K_n for every
mode n (otherwise some processor would hold an empty block).

* Static gridding (Sec. 4.2): one grid for the whole tree; its volume is the
  sum of the nodes' TTM volumes; the optimum is found by exhaustive search
  over the psi(P, N) ordered factorisations of P.
* Dynamic gridding (Sec. 4.3, 4.4): every node u picks a grid pi(u) for its
  input (and output); if it differs from its parent's grid the input is
  redistributed at a cost of |In(u)| words.  The optimum follows the
  bottom-up recurrence of Sec. 4.4 over (node, parent grid) pairs.

Readings (the paper's text leaves them open or garbles them):
  * the grid chosen when a node regrids minimises the node's own TTM volume
    plus its subtrees' optimal volumes (the printed argmin over the subtrees
    alone can miss the optimum of the regrid branch; brute force decides);
  * T is laid out under a grid of free choice (no redistribution at the
    root): the tree's optimum is the minimum over grids g of the sum over the
    root's children of their optima given parent grid g;
  * ties between equal volumes go to the first grid in enumeration order
    (lexicographic in (q_1, ..., q_N)).

Trees are the nested tuples of oracle.plan: ("T", kids), ("m", n, kids), ("F", n).
"""
from __future__ import annotations

import itertools
import math
from functools import lru_cache


# --------------------------------------------------------------------------
# Sec. 4.2: number of grids and their enumeration
# --------------------------------------------------------------------------
def factorize(P: int) -> dict:
    """Prime factorisation {p: e} of P >= 1 by trial division."""
    out, p, x = {}, 2, int(P)
    while p * p <= x:
        while x % p == 0:
            out[p] = out.get(p, 0) + 1
            x //= p
        p += 1
    if x > 1:
        out[x] = out.get(x, 0) + 1
    return out


def psi(P: int, N: int) -> int:
    """Ordered factorisations of P into N factors: prod_i C(e_i + N - 1, N - 1)."""
    r = 1
    for e in factorize(P).values():
        r *= math.comb(e + N - 1, N - 1)
    return r


def grids(P: int, N: int):
    """All N-tuples of positive integers with product P, lexicographic order."""
    if N == 1:
        return [(P,)]
    out = []
    for d in range(1, P + 1):
        if P % d == 0:
            for rest in grids(P // d, N - 1):
                out.append((d,) + rest)
    return out


def valid(g, K) -> bool:
    return all(q <= k for q, k in zip(g, K))


# --------------------------------------------------------------------------
# tree helpers: internal nodes with parent, mode, |In|, |Out|
# --------------------------------------------------------------------------
def internal_nodes(L, K, tree):
    """[(parent_index or -1, mode, in_card, out_card)] in depth-first order."""
    size_T = 1
    for x in L:
        size_T *= int(x)
    out = []

    def visit(node, parent, size_in):
        if node[0] == "F":
            return
        n = node[1]
        size_out = size_in // int(L[n]) * int(K[n])
        idx = len(out)
        out.append((parent, n, size_in, size_out))
        for c in node[2]:
            visit(c, idx, size_out)

    for c in tree[1]:
        visit(c, -1, size_T)
    return out


# --------------------------------------------------------------------------
# volumes of a given scheme
# --------------------------------------------------------------------------
def static_volume(L, K, tree, g) -> int:
    """Sum over internal nodes of (q_n - 1) |Out(u)| under one grid g."""
    return sum((g[n] - 1) * oc for _, n, _, oc in internal_nodes(L, K, tree))


def dynamic_volume(L, K, tree, root_grid, pi) -> int:
    """Volume of the dynamic scheme pi (grid per internal node, depth-first
    order) with T laid out under root_grid: TTM volume at every node plus
    |In(u)| wherever pi(u) differs from the grid of u's parent."""
    nodes = internal_nodes(L, K, tree)
    vol = 0
    for u, (parent, n, ic, oc) in enumerate(nodes):
        pg = root_grid if parent < 0 else pi[parent]
        vol += (pi[u][n] - 1) * oc
        if tuple(pi[u]) != tuple(pg):
            vol += ic
    return vol


# --------------------------------------------------------------------------
# optima
# --------------------------------------------------------------------------
def optimal_static(L, K, tree, P: int):
    """(volume, grid) of the best valid static grid, or None if none is valid."""
    best = None
    for g in grids(P, len(L)):
        if not valid(g, K):
            continue
        v = static_volume(L, K, tree, g)
        if best is None or v < best[0]:
            best = (v, g)
    return best


def optimal_dynamic(L, K, tree, P: int):
    """(volume, root grid, pi) of the optimal dynamic scheme by the bottom-up
    recurrence over (node, parent grid) pairs (Sec. 4.4)."""
    nodes = internal_nodes(L, K, tree)
    G = [g for g in grids(P, len(L)) if valid(g, K)]
    if not G:
        return None
    kids = [[] for _ in nodes]
    roots = []
    for u, (parent, _, _, _) in enumerate(nodes):
        (roots if parent < 0 else kids[parent]).append(u)

    @lru_cache(maxsize=None)
    def below(u, gi):
        """Optimal volume of the children subtrees of u when u's output is under G[gi]."""
        return sum(best(v, gi)[0] for v in kids[u])

    @lru_cache(maxsize=None)
    def regrid(u):
        """Best grid for u when it regrids: its TTM volume plus the subtrees."""
        _, n, _, oc = nodes[u]
        return min(range(len(G)), key=lambda gi: ((G[gi][n] - 1) * oc + below(u, gi), gi))

    @lru_cache(maxsize=None)
    def best(u, pgi):
        """(volume, chosen grid index) of subtree u given its parent's grid G[pgi]."""
        _, n, ic, oc = nodes[u]
        keep = (G[pgi][n] - 1) * oc + below(u, pgi)
        ri = regrid(u)
        move = ic + (G[ri][n] - 1) * oc + below(u, ri)
        if ri == pgi or keep <= move:
            return keep, pgi
        return move, ri

    def total(gi):
        return sum(best(u, gi)[0] for u in roots)

    g0 = min(range(len(G)), key=lambda gi: (total(gi), gi))
    pi = [None] * len(nodes)

    def assign(u, pgi):
        _, gi = best(u, pgi)
        pi[u] = G[gi]
        for v in kids[u]:
            assign(v, gi)

    for u in roots:
        assign(u, g0)
    return total(g0), G[g0], pi


def brute_dynamic(L, K, tree, P: int) -> int:
    """Minimum of dynamic_volume over every root grid and every assignment of
    valid grids to the internal nodes (tiny cases only)."""
    nodes = internal_nodes(L, K, tree)
    G = [g for g in grids(P, len(L)) if valid(g, K)]
    best = None
    for g0 in G:
        for pi in itertools.product(G, repeat=len(nodes)):
            v = dynamic_volume(L, K, tree, g0, pi)
            if best is None or v < best:
                best = v
    return best
