"""A^{-1} B for an HSS matrix A and a dense block B: the four steps of
Sec. 4.3 (implicit ULV after Chandrasekaran, Gu and Pals), taken literally.

Test infrastructure only (see ``oracle/__init__``).

Step 1  For every leaf i, a QL factorization U_i = Q_i [0; U~_i] and an
        orthogonal Z_i with Q_i^T D_i Z_i = [[D~_i11, 0], [D~_i21, D~_i22]],
        D~_i11 lower triangular (here: an LQ factorization of the leading
        rows of Q_i^T D_i).  B is replaced by Q^T B.
Step 2  A~ = Q^T A Z = A1 A2 with A1(:, I_j) = [C1, E2], A2(:, I_j) = [E1, C2]
        (C2 the last columns of each block column).  A1 = A1D + U_A V_A^T with
        A1D = blkdiag(D~_i11 (+) I); V_A^T U_A = 0 and A1D U_A = U_A give
        A1^{-1} = (I - U_A V_A^T) A1D^{-1}.  The term U_A V_A^T is the
        off-diagonal part of A1: the blocks D~_i21 inside each leaf plus an HSS
        product whose leaf row bases are U~_i and leaf column bases are the
        leading rows of Z_i^T V_i, with the same translation and core blocks.
        It is applied here literally, as a full HSS product.
Step 3  After a permutation A2 = I (+) A^_2, with A^_2 the principal submatrix
        of the kept rows/columns (HSS with leaves D~_i22, bases U~_i and the
        trailing rows of Z_i^T V_i).  Merging sibling leaves gives an HSS
        matrix of depth p-1; the procedure recurses on it.
Step 4  The solution is Z applied to the stacked (eliminated; kept) parts.

Readings where the section is silent (each listed in the design notes):
* ranks may differ per node; e_i = max(m_i - ku_i, 0) rows are eliminated and
  the kept rows/columns are the trailing ones (QL puts its zeros on top, C2 is
  the trailing block column).  With e_i = 0 the node passes through
  (Q_i = Z_i = I).
* the recursion ends with a dense LU with partial pivoting of the 1-node
  matrix (p = 0).
* the permutation of Step 3 keeps the kept unknowns leaf by leaf, so a merged
  leaf is [kept(c1); kept(c2)] in tree order.
* QL is computed as a reversed QR (J U J = Q' R' gives Q = J Q' J) and LQ as
  the QR of the transpose; signs of the factors are immaterial.

Pins (tests/test_oracle_ulv.py): LAPACK gesv on the assembled matrix
(n <= 4096), the Woodbury closed form for diag + low rank and the Thomas
algorithm for the tridiagonal family at large n, A (A^{-1} b) = b through
the oracle matvec, the special cases A = I, B-blocks = 0, p = 0, and the
structural claims of Step 1/2 (zero rows of Q^T U, triangular D~_11,
V_A^T U_A = 0).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .hss import HSS, _blkdiag
from .matvec import matvec


def ql(U: np.ndarray):
    """U = Q [0; L] with Q square orthogonal and L the trailing rows.
    Returns (Q, QtU) where QtU = Q^T U has zeros in its leading m-k rows."""
    m, k = U.shape
    if k >= m:
        return np.eye(m), U.copy()
    Qp, Rp = np.linalg.qr(U[::-1, ::-1], mode="complete")
    Q = Qp[::-1, ::-1]
    return Q, Rp[::-1, ::-1]


def lq(M: np.ndarray):
    """M = [L 0] Z^T, i.e. M Z = [L 0] with L lower triangular (rows(M) x rows(M))."""
    e, m = M.shape
    Z, R = np.linalg.qr(M.T, mode="complete")
    return Z, R[:e, :e].T


def step1_leaf(D, U, V):
    """Step 1 on one leaf.  Returns a dict of the leaf's transformed blocks."""
    m = D.shape[0]
    ku = U.shape[1]
    e = max(m - ku, 0)
    Q, QtU = ql(U)
    M = Q.T @ D
    if e > 0:
        Z, L = lq(M[:e])
    else:
        Z, L = np.eye(m), np.zeros((0, 0))
    Dt = M @ Z
    Vh = Z.T @ V
    return dict(e=e, Q=Q, Z=Z, L=L, Ut=QtU[e:], QtU=QtU, Dt=Dt,
                D21=Dt[e:, :e], D22=Dt[e:, e:], Vtop=Vh[:e], Vbot=Vh[e:])


def solve(H: HSS, B: np.ndarray) -> np.ndarray:
    """X = A^{-1} B by Steps 1-4 of Sec. 4.3 (recursive)."""
    B = np.asarray(B, dtype=np.float64)
    vec = B.ndim == 1
    if vec:
        B = B[:, None]
    X = _solve(H, B)
    return X[:, 0] if vec else X


def _solve(H: HSS, B: np.ndarray) -> np.ndarray:
    p = H.p
    if p == 0:
        return sla.lu_solve(sla.lu_factor(H.D[0]), B)
    rg = H.ranges()
    leaves = range(2 ** p - 1, 2 ** (p + 1) - 1)

    # Step 1: per-leaf QL / LQ, and Q^T B.
    f, bt = {}, {}
    for t in leaves:
        a, b = rg[t]
        f[t] = step1_leaf(H.D[t], H.U[t], H.V[t])
        bt[t] = f[t]["Q"].T @ B[a:b]

    # Step 2: A1^{-1} Q^T B = (I - U_A V_A^T) A1D^{-1} Q^T B.
    # A1D^{-1}: L^{-1} on the eliminated rows, identity on the kept rows.
    y = {}
    for t in leaves:
        e = f[t]["e"]
        y[t] = (sla.solve_triangular(f[t]["L"], bt[t][:e], lower=True) if e > 0
                else np.zeros((0, B.shape[1])))
    # U_A V_A^T applied to that vector: only the kept rows receive anything;
    # only the eliminated components (y) contribute.
    row_off, col_off = [0], [0]
    for t in leaves:
        row_off.append(row_off[-1] + H.D[t].shape[0] - f[t]["e"])
        col_off.append(col_off[-1] + f[t]["e"])
    corr_hss = HSS(row_off[-1], p, row_off, H.ku, H.kv, {},
                   {t: f[t]["Ut"] for t in leaves},
                   {t: f[t]["Vtop"] for t in leaves},
                   H.R, H.W, H.B12, H.B21, col_leaf_off=col_off)
    ycat = np.vstack([y[t] for t in leaves])
    corr = matvec(corr_hss, ycat, with_diag=False)
    g = {}
    for j, t in enumerate(leaves):
        e = f[t]["e"]
        g[t] = bt[t][e:] - f[t]["D21"] @ y[t] - corr[row_off[j]:row_off[j + 1]]

    # Step 3: merge sibling leaves of A^_2 into a depth p-1 HSS matrix, recurse.
    lvl = p - 1
    D2, U2, V2 = {}, {}, {}
    new_off = [0]
    for t in range(2 ** lvl - 1, 2 ** p - 1):
        c1, c2 = 2 * t + 1, 2 * t + 2
        f1, f2 = f[c1], f[c2]
        top = np.hstack([f1["D22"], f1["Ut"] @ H.B12[t] @ f2["Vbot"].T])
        bot = np.hstack([f2["Ut"] @ H.B21[t] @ f1["Vbot"].T, f2["D22"]])
        D2[t] = np.vstack([top, bot])
        if lvl > 0:
            U2[t] = _blkdiag(f1["Ut"], f2["Ut"]) @ H.R[t]
            V2[t] = _blkdiag(f1["Vbot"], f2["Vbot"]) @ H.W[t]
        new_off.append(new_off[-1] + D2[t].shape[0])
    nn2 = 2 ** lvl - 1
    R2 = {t: H.R[t] for t in H.R if t < nn2}
    W2 = {t: H.W[t] for t in H.W if t < nn2}
    B12 = {t: H.B12[t] for t in H.B12 if t < nn2}
    B21 = {t: H.B21[t] for t in H.B21 if t < nn2}
    nnodes2 = 2 ** (lvl + 1) - 1
    H2 = HSS(new_off[-1], lvl, new_off, H.ku[:nnodes2], H.kv[:nnodes2],
             D2, U2, V2, R2, W2, B12, B21)
    gcat = np.vstack([g[t] for t in leaves])
    xhat = _solve(H2, gcat)

    # Step 4: x_i = Z_i [y_i; x^_i].
    X = np.zeros_like(B)
    for j, t in enumerate(leaves):
        a, b = rg[t]
        kept = xhat[row_off[j]:row_off[j + 1]]
        X[a:b] = f[t]["Z"] @ np.vstack([y[t], kept])
    return X
