"""Pins of the oracle's dense-to-HSS constructor (Sec. 3.2)."""
import numpy as np
import pytest

from oracle import tree
from oracle.construct import construct
from oracle.hss import HSS
from paper_1909_07909_amd import inputs
from tests.cauchy_fixture import compress as one_sided


def test_exact_hss_matrix_recovered():
    """A matrix that is exactly HSS with ranks 5 (random generators): every
    block row and column has rank 5, so the constructor returns ranks 5 and
    the matrix to rounding."""
    lo = tree.leaf_offsets(512, 32)
    A = HSS.from_packed(inputs.synthetic_hss(lo, 5, seed=3)).dense()
    C = construct(A, lo, 1e-12)
    assert C.ku[1:] == [5] * (C.nnodes - 1) and C.kv[1:] == [5] * (C.nnodes - 1)
    assert np.max(np.abs(C.dense() - A)) <= 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("bl,bu", [(2, 3), (1, 1), (0, 4)])
def test_banded_ranks(bl, bu):
    """Banded with bandwidths (bl, bu): an exact HSS representation of rank
    bl + bu (the statement for the banded constructor in Sec. 3.2).  A block
    row couples to bl columns on its left and bu on its right: rank bu for
    the first node of a level, bl for the last, bl + bu in between; block
    columns the other way round."""
    n = 600
    lo = tree.leaf_offsets(n, 40)
    A = inputs.banded_dense(n, bl, bu, seed=5)
    C = construct(A, lo, 1e-12)
    for lev in range(1, C.p + 1):
        nodes = list(range(2 ** lev - 1, 2 ** (lev + 1) - 1))
        for t in nodes:
            first, last = t == nodes[0], t == nodes[-1]
            want_u = bu if first else (bl if last else bl + bu)
            want_v = bl if first else (bu if last else bl + bu)
            # a block with nothing to couple keeps one (zero) direction
            assert C.ku[t] == max(want_u, 1), (t, C.ku[t])
            assert C.kv[t] == max(want_v, 1), (t, C.kv[t])
    assert np.max(np.abs(C.dense() - A)) <= 1e-13 * np.max(np.abs(A))


def test_eps_zero_reproduces_any_matrix():
    """eps = 0 keeps every nonzero singular value: a random dense matrix
    (full-rank blocks) comes back to rounding."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((128, 128))
    lo = tree.leaf_offsets(128, 16)
    C = construct(A, lo, 0.0)
    assert np.max(np.abs(C.dense() - A)) <= 1e-12 * np.max(np.abs(A))
    # full-rank blocks: a node keeps min(|I_t|, n - |I_t|) directions
    rg = C.ranges()
    for t in range(1, C.nnodes):
        a, b = rg[t]
        assert C.ku[t] == C.kv[t] == min(b - a, 128 - (b - a))


def test_leaf_truncation_is_eckart_young():
    """At the leaves the kept basis is the best rank-k one: the projection
    error of the block row is its (k+1)-th singular value, below
    eps sigma_1, and the k-th lies above."""
    n, eps = 1024, 1e-8
    lo = tree.leaf_offsets(n, 64)
    A = inputs.cauchy_kernel_dense(n, seed=2)
    C = construct(A, lo, eps)
    rg = C.ranges()
    for t in range(2 ** C.p - 1, C.nnodes):
        a, b = rg[t]
        Hr = np.hstack([A[a:b, :a], A[a:b, b:]])
        s = np.linalg.svd(Hr, compute_uv=False)
        k = C.ku[t]
        U = C.U[t]
        err = np.linalg.norm(Hr - U @ (U.T @ Hr), 2)
        assert abs(err - s[k]) <= 1e-12 * s[0]
        assert s[k] <= eps * s[0] < s[k - 1]


def test_nested_bases_orthonormal():
    lo = tree.leaf_offsets(1000, 50)
    A = inputs.cauchy_kernel_dense(1000, seed=4)
    C = construct(A, lo, 1e-10)
    Ue, Ve = C.explicit_bases()
    for t in range(1, C.nnodes):
        for B in (Ue[t], Ve[t]):
            np.testing.assert_allclose(B.T @ B, np.eye(B.shape[1]), atol=1e-13)


@pytest.mark.parametrize("eps", [1e-6, 1e-10])
def test_error_and_one_sided_compressor(eps):
    """The whole error is a small multiple of eps ||A||_2 (each truncation
    discards at most eps sigma_1 of a block row or column); an independent
    compressor that truncates each side over the full block rows gets the
    same ranks within one and the same matrix to that order."""
    n = 2048
    lo = tree.leaf_offsets(n, 64)
    A = inputs.cauchy_kernel_dense(n, seed=6)
    nrm = np.linalg.norm(A, 2)
    C = construct(A, lo, eps)
    err = np.linalg.norm(C.dense() - A, 2)
    assert err <= 4 * C.p * eps * nrm
    F = HSS.from_packed(one_sided(np.ascontiguousarray(A), lo, tol=eps))
    assert np.max(np.abs(np.array(C.ku[1:]) - np.array(F.ku[1:]))) <= 1
    assert np.max(np.abs(np.array(C.kv[1:]) - np.array(F.kv[1:]))) <= 1
    assert np.linalg.norm(C.dense() - F.dense(), 2) <= 8 * C.p * eps * nrm


def test_single_leaf():
    A = np.arange(9.0).reshape(3, 3)
    C = construct(A, [0, 3], 1e-12)
    assert C.p == 0 and np.array_equal(C.dense(), A)
