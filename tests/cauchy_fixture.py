"""Input generator for the ragged-rank parity workload: a Cauchy-like kernel
matrix compressed into HSS generators on the host.

This is the construction step that precedes the hot path (the dense
constructor of Sec. 3.2, which compresses HSS block rows and columns from the
leaves to the root by truncated SVD).  Neither the oracle nor the GPU library
uses it; both consume the generators it returns, like those of
``paper_1909_07909_amd.inputs``.

Kernel: x_i sorted uniform on [0, 1],
    A_ij = 1 / (1 + ((x_i - x_j) / 0.05)^2) + 1e-2 delta_ij.
Compression: an HSS block row A(I_t, I minus I_t) keeps its left singular
directions with sigma > tol * sigma_1; at an internal node the block row is
expressed in the children's bases first, so the kept directions are the
translation operator R_t (likewise W_t for block columns).  Core blocks are
the projections of the sibling blocks onto the (orthonormal) nested bases.
"""
from __future__ import annotations

import numpy as np

from paper_1909_07909_amd.inputs import Generators, _Packer, cauchy_kernel_dense


def cauchy_matrix_for(n: int, seed: int = 1) -> np.ndarray:
    return np.ascontiguousarray(cauchy_kernel_dense(n, seed))


def _trunc_left(M: np.ndarray, tol: float) -> np.ndarray:
    if M.size == 0:
        return np.zeros((M.shape[0], 0))
    if M.shape[1] > 2 * M.shape[0]:
        # wide block: the left singular pairs of M are those of R^T, M^T = Q R
        M = np.linalg.qr(M.T, mode="r").T
    Uu, s, _ = np.linalg.svd(M, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros((M.shape[0], 0))
    k = int(np.sum(s > tol * s[0]))
    return Uu[:, :k]


def compress(A: np.ndarray, leaf_off, tol: float = 1e-10) -> Generators:
    leaf_off = np.asarray(leaf_off, dtype=np.int64)
    nleaf = leaf_off.size - 1
    p = int(round(np.log2(nleaf)))
    n = A.shape[0]
    nn = 2 ** (p + 1) - 1
    rng = [None] * nn
    for i in range(nleaf):
        rng[2 ** p - 1 + i] = (int(leaf_off[i]), int(leaf_off[i + 1]))
    for t in range(2 ** p - 2, -1, -1):
        rng[t] = (rng[2 * t + 1][0], rng[2 * t + 2][1])

    def comp_cols(t):
        a, b = rng[t]
        return np.r_[0:a, b:n]

    def off_rows(M, t):
        # the rows of M outside I_t (M has n rows)
        a, b = rng[t]
        return np.concatenate([M[:a], M[b:]])

    ku = np.zeros(nn, dtype=np.int32)
    kv = np.zeros(nn, dtype=np.int32)
    Ub, Vb, Rt, Wt = {}, {}, {}, {}
    Crow, Ccol = {}, {}          # U_t^T A(I_t, :) and (A(:, I_t) V_t)^T
    for l in range(p, 0, -1):
        for t in range(2 ** l - 1, 2 ** (l + 1) - 1):
            a, b = rng[t]
            cc = comp_cols(t)
            if l == p:
                Ub[t] = _trunc_left(off_rows(A[a:b].T, t).T, tol)
                Vb[t] = _trunc_left(off_rows(A[:, a:b], t).T, tol)
                Crow[t] = Ub[t].T @ A[a:b]
                Ccol[t] = Vb[t].T @ A[:, a:b].T
            else:
                c1, c2 = 2 * t + 1, 2 * t + 2
                Sr = np.vstack([Crow[c1], Crow[c2]])
                Sc = np.vstack([Ccol[c1], Ccol[c2]])
                Rt[t] = _trunc_left(Sr[:, cc], tol)
                Wt[t] = _trunc_left(Sc[:, cc], tol)
                Crow[t] = Rt[t].T @ Sr
                Ccol[t] = Wt[t].T @ Sc
            ku[t] = (Ub[t] if l == p else Rt[t]).shape[1]
            kv[t] = (Vb[t] if l == p else Wt[t]).shape[1]
    # explicit column bases for the core blocks
    Ve = {}
    for t in range(nn - 1, 0, -1):
        if t >= 2 ** p - 1:
            Ve[t] = Vb[t]
        else:
            c1, c2 = 2 * t + 1, 2 * t + 2
            blk = np.zeros((Ve[c1].shape[0] + Ve[c2].shape[0], Ve[c1].shape[1] + Ve[c2].shape[1]))
            blk[:Ve[c1].shape[0], :Ve[c1].shape[1]] = Ve[c1]
            blk[Ve[c1].shape[0]:, Ve[c1].shape[1]:] = Ve[c2]
            Ve[t] = blk @ Wt[t]
    pk = _Packer()
    for t in range(nn):
        a, b = rng[t]
        if t >= 2 ** p - 1:
            if p > 0:
                pk.add("U", Ub[t])
                pk.add("V", Vb[t])
            pk.add("D", A[a:b, a:b])
        else:
            c1, c2 = 2 * t + 1, 2 * t + 2
            if t != 0:
                pk.add("R", Rt[t])
                pk.add("W", Wt[t])
            (a1, b1), (a2, b2) = rng[c1], rng[c2]
            pk.add("B12", Crow[c1][:, a2:b2] @ Ve[c2])
            pk.add("B21", Crow[c2][:, a1:b1] @ Ve[c1])
    arr = pk.arrays()
    return Generators(n=n, p=p, leaf_off=leaf_off, ku=ku, kv=kv, **arr)


def cauchy_hss(n: int, leaf_off, seed: int = 1, tol: float = 1e-10):
    """(generators, dense kernel matrix) of the Cauchy-like workload."""
    A = cauchy_matrix_for(n, seed)
    return compress(A, leaf_off, tol), A
