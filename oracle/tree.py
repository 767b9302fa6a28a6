"""Cluster tree T_p (Def. 2.1) and the default splitting rule (Sec. 3.1).

Test infrastructure only (see ``oracle/__init__``).

Def. 2.1: the root is {1..n}; the 2^l nodes of level l partition {1..n} into
consecutive index sets I_i^l = {n_{i-1}^(l)+1, ..., n_i^(l)}; node I_i^l has
children I_{2i-1}^{l+1}, I_{2i}^{l+1}.  The default rule of Sec. 3.1 splits a
set {1..s} into {1..ceil(s/2)} and {ceil(s/2)+1..s} until the minimal block
size n_min is reached; with n = 2^p n_min this gives depth exactly p.  The tree
is completely balanced, so all leaves sit at one depth p, taken here as the
smallest p with ceil-halving leaves of size <= n_min, i.e. p = ceil(log2(n/n_min))
(p = 0 when n <= n_min).

Pins: the n = 8, n_min = 1 example of Fig. 1 (golden fixture), a brute-force
check of the partition properties, and the cluster-vector example
c = [2, 4, 8, 8] of Sec. 3.7.

Index sets are returned 0-based and half-open: node t covers rows
[start, stop).  Heap numbering: level l, position i (1-based) -> t = 2^l - 1 + i - 1.
"""
from __future__ import annotations

import math


def depth_for(n: int, nmin: int) -> int:
    """Depth p of the default tree: halve (ceil) until blocks have <= nmin."""
    if n <= nmin:
        return 0
    p = 0
    size = n
    while size > nmin:
        size = -(-size // 2)     # ceil(size / 2): the largest block at the next level
        p += 1
    return p


def default_tree(n: int, nmin: int) -> list[list[tuple[int, int]]]:
    """Levels l = 0..p of the default cluster tree; level l is a list of 2^l
    half-open (start, stop) pairs, left to right."""
    p = depth_for(n, nmin)
    levels = [[(0, n)]]
    for _ in range(p):
        nxt = []
        for (a, b) in levels[-1]:
            s = b - a
            half = -(-s // 2)                 # ceil(s/2) to the left child
            nxt.append((a, a + half))
            nxt.append((a + half, b))
        levels.append(nxt)
    return levels


def leaf_offsets(n: int, nmin: int) -> list[int]:
    """n_0^(p) = 0 <= n_1^(p) <= ... <= n_{2^p}^(p) = n of Def. 2.1."""
    levels = default_tree(n, nmin)
    leaves = levels[-1]
    return [leaves[0][0]] + [b for (_, b) in leaves]


def tree_from_cluster_vector(c: list[int]) -> list[list[tuple[int, int]]]:
    """Tree given by its cluster vector c = [n_1^(p), ..., n_{2^p}^(p)]
    (Sec. 3.7): leaves are the consecutive runs, upper levels are unions of
    siblings.  Empty leaves are allowed here."""
    nleaf = len(c)
    p = int(round(math.log2(nleaf)))
    if 2 ** p != nleaf:
        raise ValueError("cluster vector length must be a power of two")
    offs = [0] + list(c)
    leaves = [(offs[i], offs[i + 1]) for i in range(nleaf)]
    levels = [leaves]
    for _ in range(p):
        prev = levels[0]
        levels.insert(0, [(prev[2 * i][0], prev[2 * i + 1][1]) for i in range(len(prev) // 2)])
    return levels


def heap_ranges(levels) -> list[tuple[int, int]]:
    """Flatten the levels into heap order."""
    out = []
    for lv in levels:
        out.extend(lv)
    return out
