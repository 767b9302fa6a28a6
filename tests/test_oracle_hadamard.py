"""Pins of the oracle's HSS Hadamard product (Sec. 4.4): what the generator
algebra must assemble to, checked on dense matrices."""
import numpy as np
import pytest

from oracle import tree
from oracle.hadamard import hadamard, khatri_rao_rows, ones_hss, packed
from oracle.hss import HSS
from paper_1909_07909_amd import inputs


def _pair(n, m, ranks):
    lo = tree.leaf_offsets(n, m)
    p = int(round(np.log2(len(lo) - 1)))
    if ranks == "uniform":
        ga = inputs.synthetic_hss(lo, 4, seed=31)
        gb = inputs.synthetic_hss(lo, 3, seed=32)
    else:
        ka, va = inputs.ragged_ranks(p, seed=33, lo=2, hi=6)
        kb, vb = inputs.ragged_ranks(p, seed=34, lo=1, hi=5)
        ga = inputs.synthetic_hss_ranked(lo, ka, va, seed=35)
        gb = inputs.synthetic_hss_ranked(lo, kb, vb, seed=36)
    return HSS.from_packed(ga), HSS.from_packed(gb)


@pytest.mark.parametrize("n,m,ranks", [(512, 64, "uniform"), (600, 40, "ragged"),
                                       (257, 16, "ragged"), (64, 64, "uniform")])
def test_dense_is_elementwise_product(n, m, ranks):
    """Brute force: the assembled A o B equals dense(A) * dense(B) entry by
    entry (ragged ranks include ku != kv at most nodes)."""
    A, B = _pair(n, m, ranks)
    C = hadamard(A, B)
    ref = A.dense() * B.dense()
    got = C.dense()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    for t in range(C.nnodes):
        assert C.ku[t] == A.ku[t] * B.ku[t] and C.kv[t] == A.kv[t] * B.kv[t]


def test_ones_is_identity():
    """The all-ones matrix (rank 1 on every block) leaves A unchanged, in
    both orders, and keeps A's ranks."""
    A, _ = _pair(600, 40, "ragged")
    J = ones_hss(A.n, A.p, A.leaf_off)
    np.testing.assert_array_equal(J.dense(), np.ones((A.n, A.n)))
    for C in (hadamard(A, J), hadamard(J, A)):
        assert C.ku == A.ku and C.kv == A.kv
        np.testing.assert_allclose(C.dense(), A.dense(), rtol=0, atol=1e-13 * A.n)


def test_block_ranks_multiply():
    """Def. 2.3 on the result: every HSS block row and block column of A o B
    has rank <= ku_A ku_B (resp. kv_A kv_B), and the bound is attained for
    generic generators."""
    A, B = _pair(512, 64, "uniform")
    C = hadamard(A, B)
    M = C.dense()
    rg = C.ranges()
    n = C.n
    for t in range(1, C.nnodes):
        a, b = rg[t]
        rest = np.r_[0:a, b:n]
        for blk, k in ((M[a:b][:, rest], C.ku[t]), (M[rest][:, a:b], C.kv[t])):
            s = np.linalg.svd(blk, compute_uv=False)
            assert k == 12
            assert s.size <= k or s[k] < 1e-12 * s[0]


def test_commutes():
    A, B = _pair(600, 40, "ragged")
    np.testing.assert_allclose(hadamard(A, B).dense(), hadamard(B, A).dense(),
                               rtol=0, atol=1e-14 * 600 * 600)


def test_khatri_rao_rows_definition():
    """Row i of C .T D is kron(c_i, d_i)."""
    rng = np.random.default_rng(7)
    C = rng.standard_normal((5, 3))
    D = rng.standard_normal((5, 4))
    K = khatri_rao_rows(C, D)
    for i in range(5):
        np.testing.assert_array_equal(K[i], np.kron(C[i], D[i]))


def test_packed_round_trip():
    """packed() writes the canonical layout that HSS.from_packed reads."""
    A, B = _pair(600, 40, "ragged")
    C = hadamard(A, B)
    pk = packed(C)

    class G:
        pass
    g = G()
    g.n, g.p, g.leaf_off = C.n, C.p, np.asarray(C.leaf_off)
    g.ku, g.kv = np.asarray(C.ku), np.asarray(C.kv)
    for k, v in pk.items():
        setattr(g, k, v)
    C2 = HSS.from_packed(g)
    for nm in ("D", "U", "V", "R", "W", "B12", "B21"):
        a, b = getattr(C, nm), getattr(C2, nm)
        assert sorted(a) == sorted(b)
        for t in a:
            np.testing.assert_array_equal(a[t], b[t])


def test_rejects_different_trees():
    A, _ = _pair(512, 64, "uniform")
    B, _ = _pair(512, 32, "uniform")
    with pytest.raises(ValueError):
        hadamard(A, B)
