"""Pins of the oracle's literal A^{-1}B (Sec. 4.3)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import tree, ulv
from oracle.hss import HSS
from oracle.matvec import matvec
from paper_1909_07909_amd import inputs


def _rel(X, Xref):
    return np.max(np.linalg.norm(X - Xref, axis=0) / np.linalg.norm(Xref, axis=0))


@pytest.mark.parametrize("n,m,k,r", [(1024, 64, 8, 16), (1000, 64, 8, 3), (2048, 128, 16, 2),
                                     (96, 8, 6, 2), (4096, 64, 16, 1)])
def test_against_lapack(n, m, k, r):
    """Includes leaves with m_i = k (nothing to eliminate, e_i = 0)."""
    g = inputs.synthetic_hss(tree.leaf_offsets(n, m), k, seed=11)
    H = HSS.from_packed(g)
    A = H.dense()
    B = inputs.rhs(n, r, 12)
    ref = sla.lu_solve(sla.lu_factor(A), B)
    assert _rel(ulv.solve(H, B), ref) < 1e-13


def test_ragged_ranks_against_lapack():
    from cauchy_fixture import cauchy_hss
    n = 2048
    g, _ = cauchy_hss(n, tree.leaf_offsets(n, 128))
    H = HSS.from_packed(g)
    A = H.dense()
    B = inputs.rhs(n, 3, 13)
    X = ulv.solve(H, B)
    kappa = np.linalg.cond(A)
    assert _rel(X, np.linalg.solve(A, B)) < kappa * 1e-14
    assert np.linalg.norm(A @ X - B) / (np.linalg.norm(A, 2) * np.linalg.norm(X)) < 1e-14


@pytest.mark.parametrize("n,m,k", [(2 ** 15, 128, 6), (30001, 100, 3)])
def test_woodbury_closed_form(n, m, k):
    g, f = inputs.diag_plus_lowrank(tree.leaf_offsets(n, m), k, seed=14)
    H = HSS.from_packed(g)
    b = inputs.rhs(n, 2, 15)
    d, U, V = f["d"], f["U"], f["V"]
    Dinv_b = b / d[:, None]
    Dinv_U = U / d[:, None]
    cap = np.eye(k) + V.T @ Dinv_U
    ref = Dinv_b - Dinv_U @ np.linalg.solve(cap, V.T @ Dinv_b)
    assert _rel(ulv.solve(H, b), ref) < 1e-13


@pytest.mark.parametrize("n,m", [(2 ** 15, 128), (20000, 33)])
def test_thomas_closed_form(n, m):
    g, d = inputs.tridiagonal(tree.leaf_offsets(n, m), seed=16)
    H = HSS.from_packed(g)
    b = inputs.rhs(n, 1, 17)[:, 0]
    # Thomas algorithm (no pivoting; the matrix is diagonally dominant)
    lo, di, up = d["lower"], d["main"].copy(), d["upper"]
    rhs = b.copy()
    for i in range(1, n):
        w = lo[i - 1] / di[i - 1]
        di[i] -= w * up[i - 1]
        rhs[i] -= w * rhs[i - 1]
    x = np.zeros(n)
    x[-1] = rhs[-1] / di[-1]
    for i in range(n - 2, -1, -1):
        x[i] = (rhs[i] - up[i] * x[i + 1]) / di[i]
    np.testing.assert_allclose(ulv.solve(H, b), x, rtol=1e-12, atol=1e-13)


def test_solution_reproduces_rhs_large():
    n = 2 ** 16
    g = inputs.synthetic_hss(tree.leaf_offsets(n, 128), 16, seed=18)
    H = HSS.from_packed(g)
    b = inputs.rhs(n, 2, 19)
    x = ulv.solve(H, b)
    assert _rel(matvec(H, x), b) < 1e-14


def test_identity_gives_rhs():
    n = 2048
    g = inputs.scaled_identity(tree.leaf_offsets(n, 64), 8)
    H = HSS.from_packed(g)
    b = inputs.rhs(n, 2, 20)
    np.testing.assert_allclose(ulv.solve(H, b), b, rtol=1e-14, atol=1e-14)


def test_zero_core_is_blockwise_solve():
    n = 1024
    lo = tree.leaf_offsets(n, 64)
    g = inputs.block_diagonal(lo, 8, seed=21)
    H = HSS.from_packed(g)
    b = inputs.rhs(n, 3, 22)
    ref = np.zeros_like(b)
    for i in range(len(lo) - 1):
        t = 2 ** H.p - 1 + i
        ref[lo[i]:lo[i + 1]] = np.linalg.solve(H.D[t], b[lo[i]:lo[i + 1]])
    assert _rel(ulv.solve(H, b), ref) < 1e-14


def test_p0_dense_lu():
    g = inputs.synthetic_hss(tree.leaf_offsets(40, 64), 4, seed=23)
    H = HSS.from_packed(g)
    b = inputs.rhs(40, 2, 24)
    np.testing.assert_allclose(ulv.solve(H, b), np.linalg.solve(H.D[0], b), rtol=1e-13, atol=0)


def test_step1_structure():
    """Step 1 claims: Q^T U has zero leading rows and a lower-triangular
    trailing block; Q^T D Z has a lower-triangular leading block and a zero
    (1,2) block; Q and Z are orthogonal; the leaf is reconstructed."""
    rng = np.random.default_rng(25)
    m, k = 64, 16
    D = m * np.eye(m) + rng.standard_normal((m, m)) / 8
    U = inputs.haar_orthonormal(rng, m, k)
    V = inputs.haar_orthonormal(rng, m, k)
    f = ulv.step1_leaf(D, U, V)
    e = f["e"]
    assert e == m - k
    np.testing.assert_allclose(f["Q"].T @ f["Q"], np.eye(m), atol=1e-14)
    np.testing.assert_allclose(f["Z"].T @ f["Z"], np.eye(m), atol=1e-14)
    assert np.abs(f["QtU"][:e]).max() < 1e-14
    assert np.abs(np.triu(f["Ut"], 1)).max() < 1e-14
    Dt = f["Q"].T @ D @ f["Z"]
    assert np.abs(Dt[:e, e:]).max() < 1e-12
    assert np.abs(np.triu(Dt[:e, :e], 1)).max() < 1e-12
    np.testing.assert_allclose(Dt, f["Dt"], atol=1e-12)
    # reconstruction of the leaf
    np.testing.assert_allclose(f["Q"] @ f["Dt"] @ f["Z"].T, D, atol=1e-12)
    np.testing.assert_allclose(f["Z"] @ np.vstack([f["Vtop"], f["Vbot"]]), V, atol=1e-14)
