"""The allocation-free product (hss_matmul_noalloc) through the C ABI: its
result equals hss_matmul's (same kernels, work vectors in the library's fixed
device scratch instead of the handle's buffers) bit for bit, on two calls in
a row, the second with a smaller input, for both operators and precisions;
a product that does not fit the scratch is refused with HSS_ESCRATCH before
anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

from oracle import tree
from paper_1909_07909_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _to_dev(X, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(np.asfortranarray(X).T)).to(
        device="cuda", dtype=dtype).t()


def _noalloc(L, A, op, prec, X, Y):
    from paper_1909_07909_amd import hss
    xp, ldx = hss.colmajor(X, A.n)
    yp, ldy = hss.colmajor(Y, A.n)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.hss_matmul_noalloc(A.h, op, prec, X.shape[1], xp, ldx, yp, ldy, s)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("op", [0, 1])
def test_noalloc_matches_matmul(op, dtype):
    from paper_1909_07909_amd import hss
    L = hss.lib()
    prec = hss.F64 if dtype == torch.float64 else hss.F32
    # two calls in a row on different matrices, the second smaller (fewer
    # rows and columns): the shared scratch keeps the first call's contents
    cases = [(16384, 128, 32, 6, 61), (3001, 64, 16, 2, 62)]
    for n, m, k, r, seed in cases:
        print(f"[noalloc] n={n} k={k} r={r} op={op} {dtype}", flush=True)
        A = hss.HSSMatrix(inputs.synthetic_hss(tree.leaf_offsets(n, m), k, seed=seed))
        assert A.noalloc_max_rhs(prec) >= r
        X = _to_dev(inputs.rhs(n, r, seed + 100), dtype)
        ref = A.matmul(X, op=op)
        Y = hss.empty_colmajor(n, r, dtype)
        Y.fill_(float("nan"))
        assert _noalloc(L, A, op, prec, X, Y) == hss.HSS_OK
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)
        A.close()


def test_noalloc_one_rhs_then_wider():
    """The one-right-hand-side product (its fused kernels) and then a wider
    one on the same handle, each against hss_matmul."""
    from paper_1909_07909_amd import hss
    n = 65536
    A = hss.HSSMatrix(inputs.synthetic_hss(tree.leaf_offsets(n, 128), 32, seed=63))
    for r in (1, 8, 3):
        X = _to_dev(inputs.rhs(n, r, 64 + r))
        Y = hss.empty_colmajor(n, r, torch.float64)
        A.matmul_noalloc(X, Y)
        torch.cuda.synchronize()
        assert torch.equal(Y, A.matmul(X))
    A.close()


def test_noalloc_refuses_oversize():
    from paper_1909_07909_amd import hss
    L = hss.lib()
    n = 4096
    A = hss.HSSMatrix(inputs.synthetic_hss(tree.leaf_offsets(n, 128), 32, seed=65))
    rmax = A.noalloc_max_rhs(hss.F64)
    assert rmax >= 8
    X = torch.zeros((rmax + 1, n), dtype=torch.float64, device="cuda").t()
    Y = torch.full((rmax + 1, n), 7.0, dtype=torch.float64, device="cuda").t()
    assert _noalloc(L, A, 0, hss.F64, X, Y) == hss.HSS_ESCRATCH
    torch.cuda.synchronize()
    assert bool(torch.all(Y == 7.0))          # nothing was enqueued
    assert L.hss_matmul_noalloc_max_rhs(None, 0) == -1
    A.close()
