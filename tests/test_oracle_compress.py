"""Pins of the oracle's HSS recompression (Sec. 4.5, App. A)."""
import numpy as np
import pytest

from oracle import tree
from oracle.compress import compress, prop_a1_bound, proper_form
from oracle.hadamard import hadamard
from oracle.hss import HSS
from paper_1909_07909_amd import inputs


def _hss(n, m, k, seed, ragged=False):
    lo = tree.leaf_offsets(n, m)
    if ragged:
        p = int(round(np.log2(len(lo) - 1)))
        ku, kv = inputs.ragged_ranks(p, seed=seed, lo=3, hi=k)
        return HSS.from_packed(inputs.synthetic_hss_ranked(lo, ku, kv, seed=seed + 1))
    return HSS.from_packed(inputs.synthetic_hss(lo, k, seed=seed))


def _pad(H, extra, seed):
    """The same matrix with every rank raised by `extra`: random extra basis
    columns, zero rows and columns in the core blocks and translation
    operators, so the represented matrix is unchanged."""
    rng = np.random.default_rng(seed)
    ku = [k + extra if t else 0 for t, k in enumerate(H.ku)]
    kv = [k + extra if t else 0 for t, k in enumerate(H.kv)]
    U, V, R, W, B12, B21 = {}, {}, {}, {}, {}, {}
    for t in range(H.nnodes):
        if H.is_leaf(t):
            if t in H.U:
                U[t] = np.hstack([H.U[t], rng.standard_normal((H.U[t].shape[0], extra))])
                V[t] = np.hstack([H.V[t], rng.standard_normal((H.V[t].shape[0], extra))])
        else:
            c1, c2 = 2 * t + 1, 2 * t + 2
            if t != 0:
                for src, dst, k in ((H.R, R, H.ku), (H.W, W, H.kv)):
                    old = src[t]
                    a1, a2 = k[c1], k[c2]
                    new = rng.standard_normal((a1 + a2 + 2 * extra, k[t] + extra))
                    new[:, :k[t]] = 0.0
                    new[:a1, :k[t]] = old[:a1]
                    new[a1 + extra:a1 + extra + a2, :k[t]] = old[a1:]
                    dst[t] = new
            for src, dst, r, c in ((H.B12, B12, c1, c2), (H.B21, B21, c2, c1)):
                b = np.zeros((H.ku[r] + extra, H.kv[c] + extra))
                b[:H.ku[r], :H.kv[c]] = src[t]
                dst[t] = b
    return HSS(H.n, H.p, H.leaf_off, ku, kv, dict(H.D), U, V, R, W, B12, B21)


@pytest.mark.parametrize("n,m,k,ragged", [(1024, 64, 8, False), (900, 50, 7, True)])
def test_tau_zero_keeps_the_matrix(n, m, k, ragged):
    H = _hss(n, m, k, 41, ragged)
    A = H.dense()
    for C in (proper_form(H), compress(H, 0.0)):
        assert np.max(np.abs(C.dense() - A)) <= 1e-13 * np.max(np.abs(A))
    C = compress(H, 0.0)
    if not ragged:
        assert C.ku == H.ku and C.kv == H.kv
    # a block whose core has fewer rows than columns (ragged ranks) has
    # exactly that smaller rank; no other rank may change at tau = 0
    assert all(a <= b for a, b in zip(C.ku, H.ku)) and all(a <= b for a, b in zip(C.kv, H.kv))


def test_proper_form_orthonormal():
    """Phase 1: every explicit nested basis has orthonormal columns."""
    H = _hss(900, 50, 7, 43, ragged=True)
    P = proper_form(H)
    Ue, Ve = P.explicit_bases()
    for t in range(1, P.nnodes):
        for B in (Ue[t], Ve[t]):
            np.testing.assert_allclose(B.T @ B, np.eye(B.shape[1]), atol=1e-13)


def test_prop_a1_bound():
    """||A - A~||_2 <= 2 (sqrt(2^p) - 1)/(sqrt(2) - 1) tau at three
    tolerances; the ranks fall as tau grows (at tau = 1e-2 ||A||_2 every
    block row and column keeps one vector: the core blocks' singular values
    are at most 0.5 and the diagonal shift carries ||A||_2)."""
    H = _hss(1024, 64, 16, 45)
    A = H.dense()
    nrm = np.linalg.norm(A, 2)
    sums = []
    for rel in (1e-8, 1e-4, 1e-2):
        tau = rel * nrm
        C = compress(H, tau)
        err = np.linalg.norm(A - C.dense(), 2)
        assert err <= prop_a1_bound(H.p, tau)
        assert all(a <= b for a, b in zip(C.ku, H.ku)) and all(a <= b for a, b in zip(C.kv, H.kv))
        sums.append(sum(C.ku) + sum(C.kv))
    assert sums[0] > sums[1] > sums[2] == 2 * (H.nnodes - 1)


def test_padded_representation_recovers_rank():
    """A rank-6 matrix written with rank 10: compression at a tiny tolerance
    returns rank 6 everywhere and the same matrix."""
    H = _hss(1024, 64, 6, 47)
    Hp = _pad(H, 4, 48)
    A = H.dense()
    assert np.max(np.abs(Hp.dense() - A)) <= 1e-13 * np.max(np.abs(A))
    tau = 1e-11 * np.linalg.norm(A, 2)
    C = compress(Hp, tau)
    assert all(k == 6 for k in C.ku[1:]) and all(k == 6 for k in C.kv[1:])
    assert np.linalg.norm(C.dense() - A, 2) <= prop_a1_bound(H.p, tau)


def test_hadamard_square_rank():
    """A o A for a rank-4 A has rank-16 generators, but the Khatri-Rao column
    (a, b) equals the column (b, a): every block has rank <= 10."""
    H = _hss(1024, 64, 4, 49)
    S = hadamard(H, H)
    A = S.dense()
    tau = 1e-12 * np.linalg.norm(A, 2)
    C = compress(S, tau)
    assert max(C.ku) <= 10 and max(C.kv) <= 10 and min(C.ku[1:]) >= 1
    assert np.linalg.norm(C.dense() - A, 2) <= prop_a1_bound(S.p, tau)
