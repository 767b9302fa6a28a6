"""GPU parity at the headline size: n = 2^18, leaf 128, depth 11, k = 32, the
synthetic generators and launch configuration the benchmark times (FP64
product at 1 and 32 right-hand sides; FP32 factor + solve + FP64 refinement
and the FP64 solve, each at 1 and 32 right-hand sides).

Every output is compared in full with the FP64 oracle: the product with the
oracle's recursive product of Sec. 4.1 (relative error <= 1e-12 per column),
the solves with the oracle's literal ULV solve of Sec. 4.3 (relative
difference <= 1e-9 per column; the system is well conditioned by
construction, D_i = m I + G / sqrt(m)) and through the backward error of
Sec. 5.1 measured with the oracle's product (<= 1e-12 for FP64, <= 1e-10
after refinement).
"""
import numpy as np
import pytest

from oracle import tree
from oracle.hss import HSS
from oracle.matvec import matvec as omatvec
from oracle.norms import backward_error, norm2_power
from oracle.ulv import solve as osolve
from paper_1909_07909_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, LEAF, RANK = 2 ** 18, 128, 32


def _to_dev(X):
    return torch.from_numpy(np.ascontiguousarray(np.asfortranarray(X).T)).cuda().t()


def _to_host(t):
    return t.t().contiguous().cpu().numpy().T.astype(np.float64)


def _rel(Y, R):
    return float(np.max(np.linalg.norm(Y - R, axis=0) / np.linalg.norm(R, axis=0)))


@pytest.fixture(scope="module")
def headline():
    from paper_1909_07909_amd import hss
    g = inputs.synthetic_hss(tree.leaf_offsets(N, LEAF), RANK, seed=2)
    H = HSS.from_packed(g)
    A = hss.HSSMatrix(g)
    # one right-hand side and a block of 32, solved by the oracle together
    B = np.asfortranarray(np.hstack([inputs.rhs(N, 1, 3), inputs.rhs(N, 32, 50)]))
    Xref = osolve(H, B)
    normA = norm2_power(H, iters=5)
    yield hss, H, A, B, Xref, normA
    A.close()


@pytest.mark.parametrize("r", [1, 32])
def test_headline_matmul_f64(headline, r):
    hss, H, A, B, _, _ = headline
    print(f"[headline matmul f64] n={N} r={r}", flush=True)
    X = B[:, :1] if r == 1 else B[:, 1:]
    Y = _to_host(A.matmul(_to_dev(X)))
    assert _rel(Y, omatvec(H, X)) <= 1e-12


@pytest.mark.parametrize("r", [1, 32])
@pytest.mark.parametrize("prec", ["f64", "f32ir"])
def test_headline_solve(headline, r, prec):
    hss, H, A, B, Xref, normA = headline
    print(f"[headline solve {prec}] n={N} r={r}", flush=True)
    cols = slice(0, 1) if r == 1 else slice(1, 33)
    Bd = _to_dev(B[:, cols])
    if prec == "f64":
        A.factor(hss.F64)
        info = A.solve(Bd, prec=hss.F64, want_eta=True)
        bound = 1e-12
    else:
        A.factor(hss.F32)
        info = A.solve(Bd, prec=hss.F32, tol=1e-10, max_refine=10)
        bound = 1e-10
    X = _to_host(Bd)
    assert info["eta_max"] <= bound, info
    assert np.max(backward_error(H, X, B[:, cols], normA)) <= bound
    assert _rel(X, Xref[:, cols]) <= 1e-9
