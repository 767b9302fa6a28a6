"""Hadamard (elementwise) product of two HSS matrices, Sec. 4.4.

Test infrastructure only (see ``oracle/__init__``).

For two low-rank blocks, (U1 B1 V1^T) o (U2 B2 V2^T) =
(U1 .T U2)(B1 kron B2)(V1 .T V2)^T (eq. "hadamard"), where .T is the
transpose Khatri-Rao product: row i of C .T D is kron(c_i^T, d_i^T).  With
the nested bases of Sec. 2.2 the Khatri-Rao product passes through the
block-diagonal factor, so the translation operators of A o B are the
Kronecker products of those of A and B.  The HSS procedure of the figure
"hadamard" (right) then reads, for two matrices on the same cluster tree:

  leaves:   D = D_A o D_B,   U = U_A .T U_B,   V = V_A .T V_B
  internal: R_{U,c} = R_{U,c}^A kron R_{U,c}^B for each child c (likewise
            R_V), and every core block S = S^A kron S^B.

Readings:
* The packed layout stores R_t = [R_{U,c1}; R_{U,c2}] stacked at the parent
  (and W_t for R_V); the product is taken child block by child block, not of
  the stacked matrix.
* Ranks multiply node by node: ku_t(A o B) = ku_t(A) ku_t(B), likewise kv.
* Index order: column a kB + b of U_A .T U_B holds U_A[:, a] * U_B[:, b],
  the order numpy's ``kron`` uses for the rows and columns of R and S.

Pins (tests/test_oracle_hadamard.py): the dense assembly of the result equals
the elementwise product of the dense assemblies (brute force, uniform and
ragged ranks, ku != kv); the all-ones matrix written as a rank-1 HSS matrix
is the identity of the product; every HSS block row and column of the result
has rank <= ku_A ku_B (Def. 2.3); A o B and B o A assemble to the same matrix.
"""
from __future__ import annotations

import numpy as np

from .hss import HSS


def khatri_rao_rows(C: np.ndarray, D: np.ndarray) -> np.ndarray:
    """C .T D: row i is kron(C[i], D[i])."""
    n, q = C.shape
    m = D.shape[1]
    out = np.empty((n, q * m))
    for a in range(q):
        for b in range(m):
            out[:, a * m + b] = C[:, a] * D[:, b]
    return out


def _same_tree(A: HSS, B: HSS):
    if A.n != B.n or A.p != B.p or list(A.leaf_off) != list(B.leaf_off):
        raise ValueError("the Hadamard product needs the same cluster tree")


def hadamard(A: HSS, B: HSS) -> HSS:
    """Generators of A o B (Sec. 4.4, figure "hadamard", right)."""
    _same_tree(A, B)
    nn = A.nnodes
    ku = [A.ku[t] * B.ku[t] for t in range(nn)]
    kv = [A.kv[t] * B.kv[t] for t in range(nn)]
    D, U, V, R, W, B12, B21 = {}, {}, {}, {}, {}, {}, {}
    for t in range(nn):
        if A.is_leaf(t):
            D[t] = A.D[t] * B.D[t]
            if t in A.U:
                U[t] = khatri_rao_rows(A.U[t], B.U[t])
                V[t] = khatri_rao_rows(A.V[t], B.V[t])
        else:
            c1 = 2 * t + 1
            if t != 0:
                a1, b1 = A.ku[c1], B.ku[c1]
                R[t] = np.vstack([np.kron(A.R[t][:a1], B.R[t][:b1]),
                                  np.kron(A.R[t][a1:], B.R[t][b1:])])
                a1, b1 = A.kv[c1], B.kv[c1]
                W[t] = np.vstack([np.kron(A.W[t][:a1], B.W[t][:b1]),
                                  np.kron(A.W[t][a1:], B.W[t][b1:])])
            B12[t] = np.kron(A.B12[t], B.B12[t])
            B21[t] = np.kron(A.B21[t], B.B21[t])
    return HSS(A.n, A.p, A.leaf_off, ku, kv, D, U, V, R, W, B12, B21)


def ones_hss(n: int, p: int, leaf_off) -> HSS:
    """The n x n all-ones matrix as a rank-1 HSS matrix on the given tree
    (every basis a column of ones, every R = [1; 1], every core block 1)."""
    nn = 2 ** (p + 1) - 1
    ku = [0] + [1] * (nn - 1)
    D, U, V, R, W, B12, B21 = {}, {}, {}, {}, {}, {}, {}
    for t in range(nn):
        if t >= 2 ** p - 1:
            i = t - (2 ** p - 1)
            m = leaf_off[i + 1] - leaf_off[i]
            D[t] = np.ones((m, m))
            if p > 0:
                U[t] = np.ones((m, 1))
                V[t] = np.ones((m, 1))
        else:
            if t != 0:
                R[t] = np.ones((2, 1))
                W[t] = np.ones((2, 1))
            B12[t] = np.ones((1, 1))
            B21[t] = np.ones((1, 1))
    return HSS(n, p, leaf_off, ku, list(ku), D, U, V, R, W, B12, B21)


def packed(H: HSS) -> dict:
    """The canonical packed arrays (heap order, column-major blocks)."""
    parts = {k: [] for k in ("D", "U", "V", "R", "W", "B12", "B21")}
    for t in range(H.nnodes):
        if H.is_leaf(t):
            names = ("U", "V", "D")
        else:
            names = ("R", "W", "B12", "B21")
        for nm in names:
            blk = getattr(H, nm).get(t)
            if blk is not None:
                parts[nm].append(np.asarray(blk).ravel(order="F"))
    return {k: (np.concatenate(v) if v else np.zeros(0)) for k, v in parts.items()}
