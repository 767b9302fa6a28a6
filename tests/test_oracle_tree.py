"""Pins of the oracle's cluster tree (Def. 2.1, default split of Sec. 3.1,
cluster vectors of Sec. 3.7)."""
import os

import pytest

from oracle import tree

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows, cv = [], None
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("cluster_vector"):
                cv = [int(x) for x in line.split()[1:]]
                continue
            rows.append(tuple(int(x) for x in line.split()))
    return cv, rows


def _as_rows(levels):
    out = []
    for l, lv in enumerate(levels):
        for i, (a, b) in enumerate(lv):
            out.append((l, i + 1, a + 1, b))   # 1-based inclusive
    return out


def test_fig1_example():
    _, gold = _read("fig1_cluster_tree.txt")
    assert tree.depth_for(8, 1) == 3
    assert _as_rows(tree.default_tree(8, 1)) == gold
    assert tree.leaf_offsets(8, 1) == list(range(9))   # c = [1, ..., 8]


def test_cluster_vector_example():
    cv, gold = _read("cluster_vector_example.txt")
    assert _as_rows(tree.tree_from_cluster_vector(cv)) == gold


@pytest.mark.parametrize("n,nmin", [(1, 1), (5, 8), (8, 8), (9, 8), (100, 7), (1000, 64),
                                    (1024, 64), (16384, 128), (262144, 128), (4097, 128),
                                    (2049, 64), (32768, 64), (777, 3)])
def test_partition_properties(n, nmin):
    """Def. 2.1 checked directly: every level partitions {1..n} into
    consecutive sets, children partition their parent, the left child gets
    ceil(s/2) (Sec. 3.1), all leaves are at depth p and have <= nmin indices,
    and depth p - 1 would leave a block above nmin."""
    levels = tree.default_tree(n, nmin)
    p = len(levels) - 1
    assert p == tree.depth_for(n, nmin)
    for l, lv in enumerate(levels):
        assert len(lv) == 2 ** l
        assert lv[0][0] == 0 and lv[-1][1] == n
        for (a, b), (c, d) in zip(lv, lv[1:]):
            assert b == c
        if l < p:
            for i, (a, b) in enumerate(lv):
                (a1, b1), (a2, b2) = levels[l + 1][2 * i], levels[l + 1][2 * i + 1]
                assert a1 == a and b1 == a2 and b2 == b
                assert b1 - a1 == -(-(b - a) // 2)
    assert max(b - a for a, b in levels[-1]) <= nmin
    if p > 0:
        assert max(b - a for a, b in levels[-2]) > nmin
    # n = 2^p n_min gives depth exactly p with equal leaves (Sec. 2.1)
    if n % nmin == 0 and (n // nmin) & (n // nmin - 1) == 0:
        assert 2 ** p * nmin == n
        assert all(b - a == nmin for a, b in levels[-1])


def test_brute_force_small():
    """Exhaustive over small n, nmin: the depth is the smallest p whose
    ceil-halved leaves fit, computed by brute force from the sizes alone."""
    for n in range(1, 130):
        for nmin in range(1, 20):
            levels = tree.default_tree(n, nmin)
            p = 0
            while True:
                sizes = [n]
                for _ in range(p):
                    sizes = [s for x in sizes for s in (-(-x // 2), x // 2)]
                if max(sizes) <= nmin:
                    break
                p += 1
            assert len(levels) - 1 == p
            assert [b - a for a, b in levels[-1]] == sizes
