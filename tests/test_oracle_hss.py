"""Pins of the oracle's generator semantics and dense assembly (Sec. 2.2)."""
import numpy as np
import pytest

from oracle import tree
from oracle.hss import HSS
from paper_1909_07909_amd import inputs


def _levels(p):
    return [(l, range(2 ** l - 1, 2 ** (l + 1) - 1)) for l in range(p + 1)]


@pytest.mark.parametrize("n,m,k", [(1024, 64, 8), (512, 64, 16), (1000, 64, 8)])
def test_sibling_blocks_have_core_singular_values(n, m, k):
    """With orthonormal leaf bases and translation operators the nested bases
    are orthonormal, so every assembled sibling block U B V^T has exactly the
    singular values prescribed for B (0.5 * 10^(-j/4))."""
    g = inputs.synthetic_hss(tree.leaf_offsets(n, m), k, seed=3)
    H = HSS.from_packed(g)
    A = H.dense()
    rg = H.ranges()
    sig = 0.5 * 10.0 ** (-np.arange(k) / 4.0)
    for t in range(2 ** H.p - 1):
        (a1, b1), (a2, b2) = rg[2 * t + 1], rg[2 * t + 2]
        for blk in (A[a1:b1, a2:b2], A[a2:b2, a1:b1]):
            s = np.linalg.svd(blk, compute_uv=False)
            np.testing.assert_allclose(s[:k], sig, rtol=1e-12, atol=1e-14)
            assert np.all(s[k:] < 1e-13)


@pytest.mark.parametrize("n,m,k", [(1024, 64, 8), (768, 32, 4)])
def test_hss_block_rank(n, m, k):
    """Def. 2.3: every HSS block row A(I_t, I minus I_t) and block column has
    rank <= k."""
    g = inputs.synthetic_hss(tree.leaf_offsets(n, m), k, seed=4)
    H = HSS.from_packed(g)
    A = H.dense()
    rg = H.ranges()
    for t in range(1, H.nnodes):
        a, b = rg[t]
        rest = np.r_[0:a, b:n]
        for blk in (A[a:b][:, rest], A[rest][:, a:b]):
            s = np.linalg.svd(blk, compute_uv=False)
            assert s.size <= k or s[k] < 1e-12 * s[0]
            assert s[min(k, s.size) - 1] > 1e-10


@pytest.mark.parametrize("n,m", [(1000, 64), (64, 64), (257, 16), (8, 1)])
def test_tridiagonal_assembles_to_stencil(n, m):
    lo = tree.leaf_offsets(n, m)
    g, diag = inputs.tridiagonal(lo, seed=5)
    A = HSS.from_packed(g).dense()
    T = np.diag(diag["main"]) + np.diag(diag["upper"], 1) + np.diag(diag["lower"], -1)
    np.testing.assert_array_equal(A, T)


@pytest.mark.parametrize("n,m,k", [(1024, 64, 3), (999, 50, 5)])
def test_diag_plus_lowrank_assembles(n, m, k):
    lo = tree.leaf_offsets(n, m)
    g, f = inputs.diag_plus_lowrank(lo, k, seed=6)
    A = HSS.from_packed(g).dense()
    ref = np.diag(f["d"]) + f["U"] @ f["V"].T
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-15)


def test_packed_size_mismatch_rejected():
    g = inputs.synthetic_hss(tree.leaf_offsets(256, 32), 4, seed=0)
    g.R = g.R[:-1]
    with pytest.raises(ValueError):
        HSS.from_packed(g)


def test_generator_entry_count_formula():
    """The generator entry count of the headline workload (n = 2^18, m = 128,
    k = 32): sum over leaves of m^2 + 2mk, over non-root internal nodes of
    2 * 2k*k, over internal nodes of 2 k*k."""
    n, m, k = 2 ** 18, 128, 32
    p = tree.depth_for(n, m)
    nleaf = 2 ** p
    expect = nleaf * (m * m + 2 * m * k) + (2 ** p - 2) * 2 * (2 * k * k) + (2 ** p - 1) * 2 * k * k
    assert expect == 62_904_320
