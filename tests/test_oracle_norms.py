"""Pins of the ||A||_2 power method (Sec. 4.5) and the backward error of
Sec. 5.1."""
import numpy as np

from oracle import tree
from oracle.hss import HSS
from oracle.norms import backward_error, norm2_power
from oracle.ulv import solve
from paper_1909_07909_amd import inputs


def test_scaled_identity():
    g = inputs.scaled_identity(tree.leaf_offsets(512, 64), 4, c=3.5)
    assert abs(norm2_power(HSS.from_packed(g), iters=5) - 3.5) < 1e-14


def test_laplacian_closed_form():
    """(2, -1) tridiagonal matrix of order n: ||A||_2 = 2 + 2 cos(pi/(n+1))."""
    n = 24
    g, d = inputs.tridiagonal(tree.leaf_offsets(n, 4), seed=0)
    H = HSS.from_packed(g)
    for t in H.D:
        m = H.D[t].shape[0]
        H.D[t] = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    for t in H.B12:
        H.B12[t] = np.array([[0.0, 0.0], [-1.0, 0.0]])
        H.B21[t] = np.array([[0.0, -1.0], [0.0, 0.0]])
    exact = 2 + 2 * np.cos(np.pi / (n + 1))
    assert abs(norm2_power(H, iters=400) - exact) < 1e-9


def test_against_numpy_2norm():
    n = 1024
    g = inputs.scaled_identity(tree.leaf_offsets(n, 64), 4, c=1.0)
    H = HSS.from_packed(g)
    # one strong coupling at the root separates the top singular value
    H.B12[0] = np.diag([10.0, 0.0, 0.0, 0.0])
    H.B21[2] = np.diag([0.0, 3.0, 0.0, 0.0])
    A = H.dense()
    est = norm2_power(H, iters=200)
    ex = np.linalg.norm(A, 2)
    assert est <= ex * (1 + 1e-14)
    assert abs(est - ex) < 1e-6 * ex


def test_backward_error_special_cases():
    n = 512
    g = inputs.synthetic_hss(tree.leaf_offsets(n, 64), 8, seed=4)
    H = HSS.from_packed(g)
    b = inputs.rhs(n, 2, 5)
    nA = 70.0
    eta0 = backward_error(H, np.zeros_like(b), b, nA)
    np.testing.assert_allclose(eta0, 1.0, rtol=0, atol=4e-16)
    x = solve(H, b)
    assert backward_error(H, x, b, nA).max() < 1e-15
    delta = 1e-3
    eta = backward_error(H, (1 + delta) * x, b, nA)
    expect = delta * np.linalg.norm(b, axis=0) / (
        nA * (1 + delta) * np.linalg.norm(x, axis=0) + np.linalg.norm(b, axis=0))
    np.testing.assert_allclose(eta, expect, rtol=1e-9)
