"""GPU: the continuous-batching server completes every request to its
tolerance class, and each result equals the request solved alone within that
tolerance (both have backward error <= tol and the matrices are well
conditioned, so their difference is bounded by a small multiple of tol)."""
import numpy as np
import pytest

from oracle.hss import HSS
from oracle.matvec import matvec as omatvec

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_server_alone_vs_mix():
    from paper_1909_07909_amd import hss, serve
    specs = serve.draw_catalogue(4, seed=4, n_lo=4096, n_hi=16384)
    gens = serve.build_catalogue(specs, seed=4, workers=1)
    mats = [hss.HSSMatrix(g) for g in gens]
    for m in mats:
        m.factor(hss.F32)
    reqs = serve.poisson_requests(rate=4000.0, duration=0.02, n_mats=len(mats), seed=5)
    assert len(reqs) >= 20
    srv, wall = serve.run_stream(mats, reqs, budget_bytes=1 << 30, workers=2)
    assert not srv.errors, srv.errors
    assert len(srv.done) == len(reqs)
    assert max(srv.round_sizes) > 1          # requests really shared rounds
    for r in srv.done:
        assert r.status == 0, r
        assert r.eta.max() <= r.tol, (r.rid, r.eta.max(), r.tol)
    # alone vs in the mix
    for r in srv.done[:12]:
        A = mats[r.mat]
        B = torch.from_numpy(np.ascontiguousarray(r.B.T)).cuda().t()
        info = A.solve(B, prec=hss.F32, tol=r.tol)
        alone = B.t().contiguous().cpu().numpy().T
        assert info["eta_max"] <= r.tol
        diff = np.linalg.norm(alone - r.X, axis=0) / np.linalg.norm(alone, axis=0)
        assert diff.max() <= 10 * r.tol, (r.rid, diff.max(), r.tol)
    # one request against the oracle product
    r = srv.done[0]
    H = HSS.from_packed(gens[r.mat])
    res = r.B - omatvec(H, r.X)
    assert np.linalg.norm(res) / np.linalg.norm(r.B) < 10 * r.tol


def test_server_device_requests():
    """Device-resident request blocks: packed by device copies, results are
    views of the round's block; each equals the request solved alone."""
    from paper_1909_07909_amd import hss, serve
    specs = serve.draw_catalogue(3, seed=6, n_lo=4096, n_hi=16384)
    gens = serve.build_catalogue(specs, seed=6, workers=1)
    mats = [hss.HSSMatrix(g) for g in gens]
    for m in mats:
        m.factor(hss.F32)
    pools = serve.rhs_pools(mats, width=16, seed=9, device=True)
    reqs = serve.poisson_requests(rate=4000.0, duration=0.02, n_mats=len(mats), seed=7)
    srv, wall = serve.run_stream(mats, reqs, budget_bytes=1 << 30, workers=2, pools=pools)
    assert not srv.errors, srv.errors
    assert len(srv.done) == len(reqs)
    for r in srv.done:
        assert r.status == 0 and r.eta.max() <= r.tol, (r.rid, r.eta.max(), r.tol)
        assert isinstance(r.X, torch.Tensor) and r.X.is_cuda
    for r in srv.done[:10]:
        A = mats[r.mat]
        B = hss.empty_colmajor(A.n, r.nrhs, torch.float64).copy_(r.B)
        info = A.solve(B, prec=hss.F32, tol=r.tol)
        assert info["eta_max"] <= r.tol
        diff = torch.linalg.norm(B - r.X, dim=0) / torch.linalg.norm(B, dim=0)
        assert float(diff.max()) <= 10 * r.tol, (r.rid, float(diff.max()), r.tol)


def test_server_catalogue_lru():
    """Residency bounded by a catalogue: four matrices, room for about two;
    matrices are created and factored when a round first needs them and the
    least recently used idle ones are evicted.  Every request still meets its
    tolerance and equals the request solved alone."""
    from paper_1909_07909_amd import hss, serve
    specs = serve.draw_catalogue(4, seed=8, n_lo=4096, n_hi=16384)
    gens = serve.build_catalogue(specs, seed=8, workers=1)
    sizes = []
    for g in gens:
        A = hss.HSSMatrix(g)
        A.factor(hss.F32)
        sizes.append(A.query(hss.Q_RESIDENT_BYTES))
        A.close()
    cat = serve.Catalogue(gens, budget_bytes=int(2.2 * max(sizes)), max_cols=64)
    reqs = serve.poisson_requests(rate=3000.0, duration=0.03, n_mats=len(gens), seed=9)
    srv, wall = serve.run_stream(cat, reqs, budget_bytes=1 << 30, workers=2)
    st = cat.stats()
    assert not srv.errors, srv.errors
    assert len(srv.done) == len(reqs)
    assert st["misses"] >= len(gens) and st["evictions"] > 0, st
    # the budget holds, up to one matrix a round takes when nothing else fits
    assert st["resident_bytes"] <= st["budget_bytes"] + max(sizes), st
    for r in srv.done:
        assert r.status == 0 and r.eta.max() <= r.tol, (r.rid, r.eta.max(), r.tol)
    for r in srv.done[:8]:
        A = hss.HSSMatrix(gens[r.mat])
        A.factor(hss.F32)
        B = torch.from_numpy(np.ascontiguousarray(r.B.T)).cuda().t()
        info = A.solve(B, prec=hss.F32, tol=r.tol)
        alone = B.t().contiguous().cpu().numpy().T
        assert info["eta_max"] <= r.tol
        diff = np.linalg.norm(alone - r.X, axis=0) / np.linalg.norm(alone, axis=0)
        assert diff.max() <= 10 * r.tol, (r.rid, diff.max(), r.tol)
        A.close()
