"""HSS approximation of a dense matrix (Sec. 3.2, the dense constructor:
low-rank truncation of every HSS block row and column from the leaves to the
root, nested, SVD truncation).

Test infrastructure only (see ``oracle/__init__``).

Level by level, from the leaves up.  M denotes the matrix seen at the level
being compressed: A itself at the leaves, afterwards the reduced matrix
blkdiag(U^_t)^T A blkdiag(V^_t) over the nodes t of the level below, whose
row block t has ku_t rows and column block t has kv_t columns.

  leaves i:    U_i <- kept left singular vectors of the block row
               A(I_i, I minus I_i); V_i likewise from the block column
               A(I minus I_i, I_i)^T; D_i = A(I_i, I_i).
  level l < p: for every node t of level l with children c1, c2 (rows and
               columns of M grouped by the children's blocks):
                 B12_t = M(c1, c2), B21_t = M(c2, c1);
                 t not the root: R_t <- kept left singular vectors of the
                 block row M(c1 u c2, everything else), W_t from the block
                 column M(everything else, c1 u c2)^T.
  after a level: M <- blkdiag(R_t)^T M blkdiag(W_t) over that level's nodes
               (at the leaves blkdiag(U_i)^T A blkdiag(V_i)).

Nestedness (eq. HSS_nestedness) holds by construction: the explicit basis of
t is blkdiag(U^_c1, U^_c2) R_t.

Readings:
* A singular value is kept when it is > eps * sigma_1 of the block being
  truncated (the relative rule stated for the dense HODLR constructor of
  Sec. 3.2), at least one per block; a block that is exactly zero keeps the
  first unit vector.
* The row and the column truncations of a level both use the reduced matrix
  as it stands at the start of that level (the paper does not fix the order;
  level by level is the order every node of a level can run in parallel).

Pins (tests/test_oracle_construct.py): a matrix that is exactly HSS with
ranks k is recovered with ranks k and to rounding; a banded matrix gets the
ranks b_l + b_u stated for the banded constructor (b_u, b_l at the first and
last nodes of a level) and is reproduced exactly; eps = 0 reproduces any
matrix; at the leaves the projection error of every block row equals its
first discarded singular value (Eckart-Young) and stays below eps sigma_1;
every explicit nested basis is orthonormal; the whole error stays within a
small multiple of eps ||A||_2 and agrees with an independent one-sided
compressor (tests/cauchy_fixture.py) to that order.
"""
from __future__ import annotations

import numpy as np

from . import tree as _tree
from .hss import HSS


def _svd_left(H: np.ndarray):
    """Left singular vectors and values of H.  A wide block is first
    reduced by a QR factorization of its transpose, H^T = Q T: H = T^T Q^T
    has the left singular pairs of the small square T^T."""
    if H.shape[1] > 2 * H.shape[0]:
        H = np.linalg.qr(H.T, mode="r").T
    Us, s, _ = np.linalg.svd(H, full_matrices=False)
    return Us, s


def truncate(H: np.ndarray, eps: float, ratios=None) -> np.ndarray:
    """Left singular vectors of H kept by the rule above; ratios: optional
    list receiving sigma_j / sigma_1."""
    r = H.shape[0]
    Us, s = (np.zeros((r, 0)), np.zeros(0)) if H.shape[1] == 0 else _svd_left(H)
    if ratios is not None:
        ratios.append(s / s[0] if s.size and s[0] > 0 else np.zeros(0))
    if s.size == 0 or s[0] == 0.0:
        e = np.zeros((r, 1))
        e[0, 0] = 1.0
        return e
    k = max(1, int(np.sum(s > eps * s[0])))
    return Us[:, :k]


def construct(A: np.ndarray, leaf_off, eps: float, record=None) -> HSS:
    """The HSS approximation of the dense n x n matrix A on the tree with
    these leaf offsets.  record: optional dict receiving sigma_j / sigma_1 of
    every truncated block, keyed by ("u" | "v", heap id)."""
    lo = [int(x) for x in leaf_off]
    nleaf = len(lo) - 1
    p = int(round(np.log2(nleaf)))
    n = A.shape[0]
    nn = 2 ** (p + 1) - 1
    rg = _tree.heap_ranges(_tree.tree_from_cluster_vector(lo[1:]))
    ku, kv = [0] * nn, [0] * nn
    D, U, V, R, W, B12, B21 = {}, {}, {}, {}, {}, {}, {}

    def trunc(side, t, H):
        ratios = [] if record is not None else None
        Q = truncate(H, eps, ratios)
        if record is not None:
            record[(side, t)] = ratios[0]
        return Q

    leaf0 = 2 ** p - 1
    for t in range(leaf0, nn):
        a, b = rg[t]
        D[t] = A[a:b, a:b].copy()
    if p == 0:
        return HSS(n, p, lo, ku, kv, D, U, V, R, W, B12, B21)
    # leaves: block rows and columns of A
    for t in range(leaf0, nn):
        a, b = rg[t]
        out = np.r_[0:a, b:n]
        Hr = A[a:b][:, out]
        Hc = A[:, a:b][out].T
        U[t] = trunc("u", t, Hr)
        V[t] = trunc("v", t, Hc)
        ku[t], kv[t] = U[t].shape[1], V[t].shape[1]
    # reduced matrix of the leaf level: blocks U_i^T A(I_i, I_j) V_j
    leaves = list(range(leaf0, nn))
    M = _reduce_first(A, rg, leaves, U, V)
    for lev in range(p - 1, -1, -1):
        below = list(range(2 ** (lev + 1) - 1, 2 ** (lev + 2) - 1))
        ro = _offsets([ku[t] for t in below])
        co = _offsets([kv[t] for t in below])
        nodes = list(range(2 ** lev - 1, 2 ** (lev + 1) - 1))
        Rl, Wl = [], []
        for t in nodes:
            c1, c2 = 2 * t + 1, 2 * t + 2
            j1, j2 = c1 - below[0], c2 - below[0]
            r1, r2 = slice(ro[j1], ro[j1 + 1]), slice(ro[j2], ro[j2 + 1])
            s1, s2 = slice(co[j1], co[j1 + 1]), slice(co[j2], co[j2 + 1])
            B12[t] = M[r1, s2].copy()
            B21[t] = M[r2, s1].copy()
            if t == 0:
                continue
            rows = slice(ro[j1], ro[j2 + 1])
            cols = slice(co[j1], co[j2 + 1])
            out_c = np.r_[0:co[j1], co[j2 + 1]:co[-1]]
            out_r = np.r_[0:ro[j1], ro[j2 + 1]:ro[-1]]
            Hr = M[rows][:, out_c]
            Hc = M[:, cols][out_r].T
            R[t] = trunc("u", t, Hr)
            W[t] = trunc("v", t, Hc)
            ku[t], kv[t] = R[t].shape[1], W[t].shape[1]
            Rl.append(R[t])
            Wl.append(W[t])
        if lev > 0:
            M = _blkdiag_list(Rl).T @ M @ _blkdiag_list(Wl)
    return HSS(n, p, lo, ku, kv, D, U, V, R, W, B12, B21)


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(int)


def _blkdiag_list(blocks):
    rows = sum(b.shape[0] for b in blocks)
    cols = sum(b.shape[1] for b in blocks)
    out = np.zeros((rows, cols))
    i = j = 0
    for b in blocks:
        out[i:i + b.shape[0], j:j + b.shape[1]] = b
        i += b.shape[0]
        j += b.shape[1]
    return out


def _reduce_first(A, rg, leaves, U, V):
    """blkdiag(U_i)^T A blkdiag(V_j), block by block."""
    ro = _offsets([U[t].shape[1] for t in leaves])
    co = _offsets([V[t].shape[1] for t in leaves])
    M = np.zeros((ro[-1], co[-1]))
    for i, t in enumerate(leaves):
        a, b = rg[t]
        for j, s in enumerate(leaves):
            c, d = rg[s]
            M[ro[i]:ro[i + 1], co[j]:co[j + 1]] = U[t].T @ A[a:b, c:d] @ V[s]
    return M
