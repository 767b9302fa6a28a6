"""HIP graph capture of the HSS product: the product's launches (one
right-hand side: the up pass with the leaves' D X, the down pass, U y^; 2-8:
the mailbox up pass with D X on the handle's side stream; wider: the
per-level kernels) record no memset and no host synchronisation (arrival
counters are never reset, mailboxes are emptied by their readers), so a
product captured once replays to the eager result.  Each graph is replayed
several times, with eager products and synchronisations between replays, and
every replay must equal the eager result bit for bit.
"""
import numpy as np
import pytest

from oracle import tree
from paper_1909_07909_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _to_dev(X):
    return torch.from_numpy(np.ascontiguousarray(np.asfortranarray(X).T)).cuda().t()


@pytest.mark.parametrize("r", [1, 4, 16])
def test_product_graph_replays(r):
    from paper_1909_07909_amd import hss
    n, m, k = 8192, 128, 32
    print(f"[graph product] n={n} k={k} r={r}", flush=True)
    A = hss.HSSMatrix(inputs.synthetic_hss(tree.leaf_offsets(n, m), k, seed=41))
    X = _to_dev(inputs.rhs(n, r, 42))
    X2 = _to_dev(inputs.rhs(n, r, 43))
    Y = hss.empty_colmajor(n, r, torch.float64)
    Y2 = hss.empty_colmajor(n, r, torch.float64)
    A.matmul(X, Y)                      # workspaces allocated before the capture
    A.matmul(X2, Y2)
    torch.cuda.synchronize()
    ref, ref2 = Y.clone(), Y2.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        A.matmul(X, Y)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        A.matmul(X, Y)
    torch.cuda.synchronize()
    for _ in range(4):
        Y.fill_(0.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)
        A.matmul(X2, Y2)                # eager product between replays
        torch.cuda.synchronize()
        assert torch.equal(Y2, ref2)
    del g
    A.close()
