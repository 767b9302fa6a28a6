"""Pins of the oracle's four-step HSS product (Sec. 4.1)."""
import numpy as np
import pytest

from oracle import tree
from oracle.hss import HSS
from oracle.matvec import matvec
from paper_1909_07909_amd import inputs


def _rel(Y, Yref):
    return np.max(np.linalg.norm(Y - Yref, axis=0) / np.linalg.norm(Yref, axis=0))


@pytest.mark.parametrize("n,m,k,r", [(1024, 64, 8, 16), (1000, 64, 8, 3), (4096, 128, 16, 2),
                                     (200, 16, 4, 1)])
@pytest.mark.parametrize("op", ["N", "T"])
def test_against_dense(n, m, k, r, op):
    g = inputs.synthetic_hss(tree.leaf_offsets(n, m), k, seed=7)
    H = HSS.from_packed(g)
    A = H.dense()
    X = inputs.rhs(n, r, 8)
    ref = (A if op == "N" else A.T) @ X
    assert _rel(matvec(H, X, op), ref) < 1e-14


def test_ragged_ranks_against_dense():
    from cauchy_fixture import cauchy_hss
    n = 2048
    g, K = cauchy_hss(n, tree.leaf_offsets(n, 128))
    assert len(set(g.ku[1:].tolist())) > 1           # ranks really vary
    H = HSS.from_packed(g)
    A = H.dense()
    X = inputs.rhs(n, 4, 9)
    for op, M in (("N", A), ("T", A.T)):
        assert _rel(matvec(H, X, op), M @ X) < 1e-14


def test_p0_is_dense_block():
    g = inputs.synthetic_hss(tree.leaf_offsets(50, 64), 4, seed=1)
    assert g.p == 0
    H = HSS.from_packed(g)
    X = inputs.rhs(50, 3, 2)
    np.testing.assert_allclose(matvec(H, X), H.D[0] @ X, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,m,k", [(2 ** 16, 128, 8), (100000, 100, 4)])
def test_diag_plus_lowrank_closed_form(n, m, k):
    g, f = inputs.diag_plus_lowrank(tree.leaf_offsets(n, m), k, seed=2)
    H = HSS.from_packed(g)
    X = inputs.rhs(n, 3, 3)
    ref = f["d"][:, None] * X + f["U"] @ (f["V"].T @ X)
    assert _rel(matvec(H, X), ref) < 1e-14
    refT = f["d"][:, None] * X + f["V"] @ (f["U"].T @ X)
    assert _rel(matvec(H, X, "T"), refT) < 1e-14


@pytest.mark.parametrize("n,m", [(2 ** 16, 128), (50001, 37)])
def test_tridiagonal_stencil(n, m):
    g, d = inputs.tridiagonal(tree.leaf_offsets(n, m), seed=3)
    H = HSS.from_packed(g)
    x = inputs.rhs(n, 1, 4)[:, 0]
    ref = d["main"] * x
    ref[:-1] += d["upper"] * x[1:]
    ref[1:] += d["lower"] * x[:-1]
    np.testing.assert_allclose(matvec(H, x), ref, rtol=1e-15, atol=1e-15)
    refT = d["main"] * x
    refT[:-1] += d["lower"] * x[1:]
    refT[1:] += d["upper"] * x[:-1]
    np.testing.assert_allclose(matvec(H, x, "T"), refT, rtol=1e-15, atol=1e-15)


def test_adjoint_identity_and_linearity():
    n = 2 ** 15
    g = inputs.synthetic_hss(tree.leaf_offsets(n, 128), 16, seed=5)
    H = HSS.from_packed(g)
    x = inputs.rhs(n, 1, 6)[:, 0]
    y = inputs.rhs(n, 1, 7)[:, 0]
    lhs = y @ matvec(H, x)
    rhs = matvec(H, y, "T") @ x
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    a, b = 0.3, -1.7
    np.testing.assert_allclose(matvec(H, a * x + b * y), a * matvec(H, x) + b * matvec(H, y),
                               rtol=1e-13, atol=1e-11)
