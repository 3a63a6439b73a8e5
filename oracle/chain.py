"""Matrix-chain parenthesisations and their costs (test infrastructure).

A chain M_1 ... M_L with M_i of size p_{i-1} x p_i can be evaluated in any
bracketing without changing the result in exact arithmetic (the associativity
that lets the paper evaluate A*B*C*D right-to-left, Sec. II, expression (6) of
Sec. III). This module enumerates every bracketing by brute force (there are
Catalan(L-1) of them), counts multiply-adds, and applies the paper's own rule:
multiply the adjacent pair whose product has the fewest elements first, then
repeat on the shortened chain (Sec. II, the A*B*C*D discussion).

A tree is either an int (leaf index) or a tuple (left, right).

Readings where the paper is silent:
* "smallest matrix" means fewest elements (rows x cols);
* ties between pairs go to the leftmost pair;
* a pair of one operand and its own transpose (same storage) may be costed as
  a symmetric rank-k update, n(n+1)/2 * k multiply-adds instead of n*n*k
  (Sec. II, the A*A^T discussion), when ``sym_pairs`` names that pair.
"""
from __future__ import annotations

from functools import lru_cache


def trees(lo: int, hi: int) -> list:
    """All full binary trees over leaves lo..hi (inclusive)."""
    if lo == hi:
        return [lo]
    out = []
    for split in range(lo, hi):
        for left in trees(lo, split):
            for right in trees(split + 1, hi):
                out.append((left, right))
    return out


def span(tree) -> tuple:
    if isinstance(tree, int):
        return tree, tree
    return span(tree[0])[0], span(tree[1])[1]


def tree_cost(tree, dims, sym_pairs=frozenset()) -> int:
    """Multiply-adds to evaluate ``tree``; dims has L+1 entries."""
    if isinstance(tree, int):
        return 0
    (a, _), (_, b) = span(tree[0]), span(tree[1])
    k = span(tree[0])[1]
    rows, inner, cols = dims[a], dims[k + 1], dims[b + 1]
    if isinstance(tree[0], int) and isinstance(tree[1], int) and (tree[0], tree[1]) in sym_pairs:
        here = rows * (rows + 1) // 2 * inner
    else:
        here = rows * inner * cols
    return here + tree_cost(tree[0], dims, sym_pairs) + tree_cost(tree[1], dims, sym_pairs)


def brute_force_min(dims, sym_pairs=frozenset()) -> tuple:
    """(min cost, list of all trees reaching it) over every bracketing."""
    n = len(dims) - 1
    best, arg = None, []
    for t in trees(0, n - 1):
        c = tree_cost(t, dims, sym_pairs)
        if best is None or c < best:
            best, arg = c, [t]
        elif c == best:
            arg.append(t)
    return best, arg


def left_to_right(n: int):
    t = 0
    for i in range(1, n):
        t = (t, i)
    return t


def right_to_left(n: int):
    t = n - 1
    for i in range(n - 2, -1, -1):
        t = (i, t)
    return t


def greedy_smallest_result(dims) -> tuple:
    """The paper's rule: repeatedly multiply the adjacent pair with the smallest
    result (leftmost on ties). Returns (tree, cost)."""
    items = [(i, dims[i], dims[i + 1]) for i in range(len(dims) - 1)]
    cost = 0
    while len(items) > 1:
        best = None
        for j in range(len(items) - 1):
            size = items[j][1] * items[j + 1][2]
            if best is None or size < best[0]:
                best = (size, j)
        j = best[1]
        (ta, ra, ka), (tb, _, cb) = items[j], items[j + 1]
        cost += ra * ka * cb
        items[j:j + 2] = [((ta, tb), ra, cb)]
    return items[0][0], cost


@lru_cache(maxsize=None)
def catalan(n: int) -> int:
    if n <= 1:
        return 1
    return sum(catalan(i) * catalan(n - 1 - i) for i in range(n))


def roofline_time(tree, dims, esz, peak_flops, bandwidth, sym_pairs=frozenset()) -> float:
    """Seconds to evaluate ``tree`` on a machine where each product takes
    the longer of its flops at ``peak_flops`` and its bytes at ``bandwidth``
    (the roofline): 2 flops per multiply-add, each operand read once and the
    result written once, ``esz`` bytes per element. A symmetric pair (see
    ``tree_cost``) does n(n+1) k flops and reads its one operand once. Not in
    the paper: the cost model of a planner variant beside the multiply-add
    count."""
    if isinstance(tree, int):
        return 0.0
    (a, _), (_, b) = span(tree[0]), span(tree[1])
    k = span(tree[0])[1]
    rows, inner, cols = dims[a], dims[k + 1], dims[b + 1]
    if isinstance(tree[0], int) and isinstance(tree[1], int) and (tree[0], tree[1]) in sym_pairs:
        flops = rows * (rows + 1) * inner
        elems = rows * inner + rows * cols
    else:
        flops = 2 * rows * inner * cols
        elems = rows * inner + inner * cols + rows * cols
    here = max(flops / peak_flops, elems * esz / bandwidth)
    return (here + roofline_time(tree[0], dims, esz, peak_flops, bandwidth, sym_pairs)
            + roofline_time(tree[1], dims, esz, peak_flops, bandwidth, sym_pairs))


def brute_force_min_time(dims, esz, peak_flops, bandwidth, sym_pairs=frozenset()) -> tuple:
    """(min roofline time, the trees within 1e-12 of it) over every bracketing."""
    n = len(dims) - 1
    times = [(roofline_time(t, dims, esz, peak_flops, bandwidth, sym_pairs), t)
             for t in trees(0, n - 1)]
    best = min(c for c, _ in times)
    return best, [t for c, t in times if c <= best * (1 + 1e-12)]
