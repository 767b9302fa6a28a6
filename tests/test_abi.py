"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol of include/hss.h, its plan is bit-exact against the oracle's
cluster tree, and invalid arguments are rejected before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import tree as otree
from paper_1909_07909_amd import hss, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "hss.h")).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(hss_\w+)\s*\(", txt, re.M)))


def test_exports_every_declared_symbol():
    L = hss.lib()
    declared = _header_symbols()
    assert len(declared) >= 13
    assert sorted(declared) == sorted(hss.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("n,nmin", [(8, 1), (1, 1), (5, 8), (1000, 64), (262144, 128),
                                    (4097, 128), (777, 3), (16384, 128), (2 ** 20, 128),
                                    (1048575, 128), (5000, 64)])
def test_plan_tree_bit_exact(n, nmin):
    assert hss.plan_depth(n, nmin) == otree.depth_for(n, nmin)
    lo = hss.plan_leaf_offsets(n, nmin)
    assert lo.dtype == np.int64
    assert lo.tolist() == otree.leaf_offsets(n, nmin)


@pytest.mark.parametrize("n,nmin", [(8, 1), (1000, 64), (4097, 128)])
def test_plan_node_ranges_bit_exact(n, nmin):
    lo = otree.leaf_offsets(n, nmin)
    p = otree.depth_for(n, nmin)
    ku, kv = inputs.uniform_ranks(p, 1)
    start, size = hss.plan_node_ranges(n, p, lo, ku, kv)
    ref = otree.heap_ranges(otree.default_tree(n, nmin))
    assert start.tolist() == [a for a, _ in ref]
    assert size.tolist() == [b - a for a, b in ref]


def test_invalid_arguments_rejected_on_host():
    L = hss.lib()
    g = inputs.synthetic_hss(otree.leaf_offsets(256, 32), 4, seed=0)
    td, keep = hss._tree(g.n, g.p, g.leaf_off, g.ku, g.kv)
    arrs = [np.ascontiguousarray(getattr(g, k)) for k in ("D", "U", "V", "R", "W", "B12", "B21")]
    gh = hss.GenHost(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs])
    h = C.c_void_p()
    assert L.hss_create(C.byref(td), C.byref(gh), None, None, None) == -5
    assert L.hss_create(None, C.byref(gh), None, None, C.byref(h)) == -1
    assert L.hss_create(C.byref(td), None, None, None, C.byref(h)) == -2
    # non-increasing leaf offsets (empty leaf)
    bad = np.array(g.leaf_off)
    bad[1] = 0
    tdb, kb = hss._tree(g.n, g.p, bad, g.ku, g.kv)
    assert L.hss_create(C.byref(tdb), C.byref(gh), None, None, C.byref(h)) == -1
    # leaf larger than the kernels take
    lo = otree.leaf_offsets(1024, 256)
    ku, kv = inputs.uniform_ranks(2, 4)
    tdl, kl = hss._tree(1024, 2, lo, ku, kv)
    assert L.hss_create(C.byref(tdl), C.byref(gh), None, None, C.byref(h)) == hss.HSS_EUNSUP
    # rank above the maximum
    ku2 = np.array(g.ku)
    ku2[3] = 65
    tdr, kr = hss._tree(g.n, g.p, g.leaf_off, ku2, g.kv)
    assert L.hss_create(C.byref(tdr), C.byref(gh), None, None, C.byref(h)) == hss.HSS_EUNSUP
    # missing generator array
    gh2 = hss.GenHost(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs])
    gh2.R = C.POINTER(C.c_double)()
    assert L.hss_create(C.byref(td), C.byref(gh2), None, None, C.byref(h)) == -2
    # NULL handle everywhere
    assert L.hss_matmul(None, 0, 0, 1, None, 1, None, 1, None) == -1
    assert L.hss_ulv_factor(None, 0, None) == -1
    assert L.hss_ulv_solve(None, 1, None, 1, None, None, None) == -1
    assert L.hss_destroy(None) == 0
    assert hss.status_str(hss.HSS_ENOCONV).startswith("refinement")
