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


def test_product_graph_survives_wider_calls():
    """A graph captured from a 4-column product keeps working after later
    calls on the same handle needed wider work buffers (a 64-column product
    and a 64-column refined solve): the buffers they replaced are kept."""
    from paper_1909_07909_amd import hss
    n, m, k, r = 4096, 128, 16, 4
    A = hss.HSSMatrix(inputs.synthetic_hss(tree.leaf_offsets(n, m), k, seed=44))
    X = _to_dev(inputs.rhs(n, r, 45))
    Y = hss.empty_colmajor(n, r, torch.float64)
    A.matmul(X, Y)
    torch.cuda.synchronize()
    ref = Y.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        A.matmul(X, Y)
    torch.cuda.synchronize()
    Xw = _to_dev(inputs.rhs(n, 64, 46))
    A.matmul(Xw)
    A.factor(hss.F32)
    A.solve(_to_dev(inputs.rhs(n, 64, 47)), prec=hss.F32, tol=1e-10)
    torch.cuda.synchronize()
    for _ in range(3):
        Y.fill_(0.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)
    del g
    A.close()


@pytest.mark.parametrize("r,max_refine", [(1, 2), (8, 3)])
def test_fresh_refined_solve_graph(r, max_refine):
    """A whole fresh-system step (FP32 factorization, FP32 solve, FP64
    residuals and gated FP32 corrections up to max_refine, the device-written
    report) captured once and replayed: the refinement steps are gated on the
    device, so the step has no host synchronisation.  Every replay must give
    the eager solution and report bit for bit."""
    from paper_1909_07909_amd import hss
    n, m, k = 8192, 128, 32
    print(f"[graph fresh step] n={n} k={k} r={r} max_refine={max_refine}", flush=True)
    A = hss.HSSMatrix(inputs.synthetic_hss(tree.leaf_offsets(n, m), k, seed=48))
    B0 = _to_dev(inputs.rhs(n, r, 49))
    B = B0.clone()
    rep = hss.SolveReport(r)

    def step():
        B.copy_(B0)
        A.factor(hss.F32)
        A.solve(B, prec=hss.F32, tol=1e-10, max_refine=max_refine, sync=False, report=rep)

    step()                                  # eager: sizes every work buffer
    torch.cuda.synchronize()
    ref_x, ref_rep = B.clone(), rep.result()
    assert ref_rep["status"] == 0 and ref_rep["iters"] == 1 and ref_rep["eta_max"] <= 1e-10
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    Bo = _to_dev(inputs.rhs(n, r, 50))
    for _ in range(4):
        B.fill_(0.0)
        rep.buf.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(B, ref_x)
        got = rep.result()
        assert np.array_equal(got["eta"], ref_rep["eta"])
        assert {k: got[k] for k in ("eta_max", "iters", "status", "norm2")} == \
               {k: ref_rep[k] for k in ("eta_max", "iters", "status", "norm2")}
        # eager work on the handle between replays
        A.solve(Bo.clone(), prec=hss.F32, tol=1e-10)
        torch.cuda.synchronize()
    del g
    A.close()


def test_batched_fresh_solve_graph():
    """Batched factorization and refined solve of uneven instances (one launch
    per tree level across them, device-gated refinement) captured once and
    replayed: the batched calls reuse their device task tables when the tables
    equal an earlier call's (an eager call on the capture stream first), so
    the graph holds no upload; every replay equals the eager solution bit for
    bit and its report up to the order of the norm sums."""
    from paper_1909_07909_amd import hss
    sizes = [(2048, 8), (3200, 16), (4096, 24), (1600, 8)]
    gens = [inputs.synthetic_hss(tree.leaf_offsets(n, 64), k, seed=90 + j)
            for j, (n, k) in enumerate(sizes)]
    mats = [hss.HSSMatrix(g) for g in gens]
    r = 4
    B0 = [_to_dev(inputs.rhs(g.n, r, 95 + j)) for j, g in enumerate(gens)]
    Bs = [b.clone() for b in B0]
    reps = [hss.SolveReport(r) for _ in mats]
    cs = torch.cuda.Stream()

    def step():
        for b, b0 in zip(Bs, B0):
            b.copy_(b0)
        hss.batch_factor(mats, hss.F32, stream=cs)
        hss.batch_solve(mats, Bs, prec=hss.F32, tol=1e-10, max_refine=2, stream=cs, sync=False,
                        reports=reps)

    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        step()
    cs.synchronize()
    ref_x = [b.clone() for b in Bs]
    ref_r = [rp.result() for rp in reps]
    assert all(x["status"] == 0 and x["iters"] == 1 and x["eta_max"] <= 1e-10 for x in ref_r)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        step()
    torch.cuda.synchronize()
    for _ in range(3):
        for b in Bs:
            b.fill_(0.0)
        for rp in reps:
            rp.buf.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for b, x in zip(Bs, ref_x):
            assert torch.equal(b, x)
        for rp, want in zip(reps, ref_r):
            got = rp.result()
            # the residual norms are sums of per-block atomics: equal up to
            # the order of those additions
            np.testing.assert_allclose(got["eta"], want["eta"], rtol=1e-12, atol=0)
            assert got["iters"] == want["iters"] and got["status"] == want["status"]
        # eager batched work between replays (other blocks, same handles)
        hss.batch_solve(mats, [b0.clone() for b0 in B0], prec=hss.F32, tol=1e-10)
        torch.cuda.synchronize()
    del g
    for m in mats:
        m.close()
