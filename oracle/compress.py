"""HSS recompression (Sec. 4.5 "Recompression" and App. A).

Test infrastructure only (see ``oracle/__init__``).

Given an HSS matrix A and a tolerance tau, build an HSS matrix on the same
tree with ranks as small as the truncation allows.  Two phases:

Phase 1, proper form (bottom-up): every basis gets orthonormal columns.
  leaves:      U_i = Q T^U_i (thin QR), U_i <- Q; likewise V_i, T^V_i.
  internal t:  [T^U_c1 R_t,1; T^U_c2 R_t,2] = Q T^U_t, R_t <- Q (t not the
               root); likewise W_t with the T^V of the children;
               B12_t <- T^U_c1 B12_t (T^V_c2)^T, B21_t <- T^U_c2 B21_t (T^V_c1)^T.
  A is unchanged; a rank becomes min(rows, columns) of its QR.

Phase 2 (top-down, levels l = 1..p): for the children c_1, c_2 of every
node i of level l - 1, the HSS block row of c_h is
U_{c_h} [S_h | R_{i,h} W_i] times a matrix with orthonormal columns, where
S_1 = B12_i, S_2 = B21_i, R_{i,h} is the child block of R_i, and W_i is the
diagonal of the singular values kept at i on the row side (no second block
when i is the root).  A truncated SVD
[S_h | R_{i,h} W_i] ~ Uh diag(s_h) Vh^T, keeping the singular values above
tau, gives the new basis U_{c_h} Uh.  The block columns are treated the
same way with V, W and the transposed core blocks: [S'_h | W_{i,h} W'_i] with
S'_1 = B21_i^T, S'_2 = B12_i^T gives Vh'.  Then
  B12_i <- U1^T B12_i V2',  B21_i <- U2^T B21_i V1',
  R_{i,h} <- Uh^T R_{i,h},  W_{i,h} <- Vh'^T W_{i,h},
  child c_h internal: R_{c_h} <- R_{c_h} Uh, W_{c_h} <- W_{c_h} Vh';
  child c_h a leaf:   U_{c_h} <- U_{c_h} Uh,  V_{c_h} <- V_{c_h} Vh'.
The singular values s_h stand in for the next level's W (the right
orthonormal factor changes no left singular vector).

Readings:
* Both SVDs of a child (row and column side) are taken from the core blocks
  as they stand before either update of that level; the paper only says the
  block columns are handled "analogously".
* A singular value is kept when it is > tau; at least one is kept at every
  node whose rank was positive (a node of rank 0 stays 0), so no basis
  becomes empty.
* Prop. A.1 states ||A - A~||_2 <= 2 (sqrt(2^p) - 1)/(sqrt(2) - 1) tau, while
  the sum in its proof, 2 sqrt(2^l) tau over l = 1..p, is sqrt(2) times
  that.  The tests check the stated (smaller) bound.

Pins (tests/test_oracle_compress.py): tau = 0 returns A to rounding;
Prop. A.1 on dense assemblies; the proper form has orthonormal nested bases;
a rank-k matrix padded to a rank-2k representation (zero columns in the
cores) compresses back to rank k; the Hadamard square of a rank-k matrix
(Sec. 4.4) compresses to rank <= k (k + 1) / 2 (its Khatri-Rao columns are
symmetric in the two factors).
"""
from __future__ import annotations

import numpy as np

from .hss import HSS


def _qr(M):
    """Thin QR with min(rows, cols) columns of Q."""
    Q, T = np.linalg.qr(M, mode="reduced")
    return Q, T


def proper_form(H: HSS) -> HSS:
    """Phase 1: the same matrix with orthonormal leaf bases and translation
    operators (bottom-up QR)."""
    nn, p = H.nnodes, H.p
    U, V, R, W = {}, {}, {}, {}
    TU, TV = {}, {}
    ku, kv = list(H.ku), list(H.kv)
    for t in range(nn - 1, 0, -1):
        if H.is_leaf(t):
            U[t], TU[t] = _qr(H.U[t])
            V[t], TV[t] = _qr(H.V[t])
        else:
            c1, c2 = 2 * t + 1, 2 * t + 2
            a1, b1 = H.ku[c1], H.kv[c1]
            MU = np.vstack([TU[c1] @ H.R[t][:a1], TU[c2] @ H.R[t][a1:]])
            MV = np.vstack([TV[c1] @ H.W[t][:b1], TV[c2] @ H.W[t][b1:]])
            R[t], TU[t] = _qr(MU)
            W[t], TV[t] = _qr(MV)
        ku[t], kv[t] = TU[t].shape[0], TV[t].shape[0]
    B12, B21 = {}, {}
    for t in range(2 ** p - 1):
        c1, c2 = 2 * t + 1, 2 * t + 2
        B12[t] = TU[c1] @ H.B12[t] @ TV[c2].T
        B21[t] = TU[c2] @ H.B21[t] @ TV[c1].T
    D = {t: H.D[t].copy() for t in H.D}
    return HSS(H.n, p, H.leaf_off, ku, kv, D, U, V, R, W, B12, B21)


def _truncate(M, tau, k_old, record=None, key=None):
    """Left singular vectors and values of M kept by the rule above (every
    singular value goes to record[key] when a dict is given)."""
    if M.shape[0] == 0:
        return np.zeros((0, 0)), np.zeros(0)
    Us, s, _ = np.linalg.svd(M, full_matrices=False)
    if record is not None:
        record[key] = s
    keep = int(np.sum(s > tau))
    if k_old > 0:
        keep = max(keep, 1)
    return Us[:, :keep], s[:keep]


def compress(H: HSS, tau: float, record=None) -> HSS:
    """Recompression with truncation tolerance tau (App. A), on a copy.
    record: optional dict that receives every SVD's singular values, keyed
    by ("u" or "v", child heap id)."""
    P = proper_form(H)
    nn, p = P.nnodes, P.p
    U = {t: P.U[t].copy() for t in P.U}
    V = {t: P.V[t].copy() for t in P.V}
    R = {t: P.R[t].copy() for t in P.R}
    W = {t: P.W[t].copy() for t in P.W}
    B12 = {t: P.B12[t].copy() for t in P.B12}
    B21 = {t: P.B21[t].copy() for t in P.B21}
    ku, kv = list(P.ku), list(P.kv)
    su, sv = {}, {}          # kept singular values (row / column side) per node
    for lev in range(1, p + 1):
        for i in range(2 ** (lev - 1) - 1, 2 ** lev - 1):
            c = (2 * i + 1, 2 * i + 2)
            a1, b1 = ku[c[0]], kv[c[0]]
            Rb = (R[i][:a1], R[i][a1:]) if i != 0 else None
            Wb = (W[i][:b1], W[i][b1:]) if i != 0 else None
            S = (B12[i], B21[i])
            St = (B21[i].T, B12[i].T)
            Uh, Vh = [], []
            for h in range(2):
                Mr = S[h] if i == 0 else np.hstack([S[h], Rb[h] * su[i]])
                Mc = St[h] if i == 0 else np.hstack([St[h], Wb[h] * sv[i]])
                u, s = _truncate(Mr, tau, ku[c[h]], record, ("u", c[h]))
                v, sc = _truncate(Mc, tau, kv[c[h]], record, ("v", c[h]))
                Uh.append(u)
                Vh.append(v)
                su[c[h]], sv[c[h]] = s, sc
            B12[i] = Uh[0].T @ B12[i] @ Vh[1]
            B21[i] = Uh[1].T @ B21[i] @ Vh[0]
            if i != 0:
                R[i] = np.vstack([Uh[0].T @ Rb[0], Uh[1].T @ Rb[1]])
                W[i] = np.vstack([Vh[0].T @ Wb[0], Vh[1].T @ Wb[1]])
            for h in range(2):
                t = c[h]
                if P.is_leaf(t):
                    U[t] = U[t] @ Uh[h]
                    V[t] = V[t] @ Vh[h]
                else:
                    R[t] = R[t] @ Uh[h]
                    W[t] = W[t] @ Vh[h]
                ku[t], kv[t] = Uh[h].shape[1], Vh[h].shape[1]
    D = {t: P.D[t].copy() for t in P.D}
    return HSS(H.n, p, H.leaf_off, ku, kv, D, U, V, R, W, B12, B21)


def prop_a1_bound(p: int, tau: float) -> float:
    """The bound of Prop. A.1 as stated: 2 (sqrt(2^p) - 1) / (sqrt(2) - 1) tau."""
    return 2.0 * (np.sqrt(2.0 ** p) - 1.0) / (np.sqrt(2.0) - 1.0) * tau
