"""The HSS matrix-vector (matrix x block) product of Sec. 4.1.

Test infrastructure only (see ``oracle/__init__``).

The four steps of the HSS procedure (Sec. 4.1 and the right half of the
figure "mat-vec"), for a block X of r columns:

  Step 1  leaves (level p): v_i^p = (V_i^(p))^T X(I_i^p),  d_i = D_i X(I_i^p);
          upward, l = p-1..1: v_i^l = (R_{V,i}^(l))^T [v_{2i-1}^{l+1}; v_{2i}^{l+1}].
  Step 2  core blocks: for every sibling pair (2i-1, 2i) of level l,
          w_{2i-1}^l = S_{2i-1,2i} v_{2i}^l,  w_{2i}^l = S_{2i,2i-1} v_{2i-1}^l.
  Step 3  downward, l = 1..p-1:
          [w_{2i-1}^{l+1}; w_{2i}^{l+1}] += R_{U,i}^(l) w_i^l.
  Step 4  leaves: Y(I_i^p) = U_i^(p) w_i^p + d_i.

Readings (the printed pseudo-code is ambiguous here):
* Step 2 runs over every level l = 1..p (sibling pairs, using the core blocks
  stored at the parent); the printed loop stops at p-1, which would drop the
  coupling between sibling leaves.  The pseudo-code overwrites v in place; the
  up values v and the down values w are kept apart here, which is what the
  in-place swap computes.
* op = 'T' multiplies by A^T: the transposed generators are D_i^T, U <-> V,
  R_U <-> R_V, and the core blocks of a pair become (B21^T, B12^T).

Pins (tests/test_oracle_matvec.py): dense assembly + BLAS at n <= 4096;
the closed forms diag(d) + U V^T and the tridiagonal stencil at large n;
p = 0 gives D X; <y, A x> = <A^T y, x>; linearity.
"""
from __future__ import annotations

import numpy as np

from .hss import HSS


def transpose(H: HSS) -> HSS:
    """Generators of A^T (same tree)."""
    D = {t: d.T.copy() for t, d in H.D.items()}
    B12 = {t: H.B21[t].T.copy() for t in H.B21}
    B21 = {t: H.B12[t].T.copy() for t in H.B12}
    return HSS(H.col_leaf_off[-1], H.p, H.col_leaf_off, H.kv, H.ku, D, dict(H.V),
               dict(H.U), dict(H.W), dict(H.R), B12, B21, col_leaf_off=H.leaf_off)


def _node(l, i):
    """Heap id of node I_i^l (i is 1-based)."""
    return 2 ** l - 1 + (i - 1)


def matvec(H: HSS, X: np.ndarray, op: str = "N", with_diag: bool = True) -> np.ndarray:
    """Y = op(A) X by the four-step procedure.  ``with_diag=False`` drops the
    D_i terms (the off-diagonal part of A only)."""
    if op == "T":
        H = transpose(H)
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    p = H.p
    rg = H.ranges()
    cg = H.col_ranges()
    Y = np.zeros((rg[0][1], X.shape[1]))
    if p == 0:
        if with_diag:
            Y[:] = H.D[0] @ X
        return Y[:, 0] if vec else Y

    v, w, d = {}, {}, {}
    # Step 1: leaves, then the upward pass with the column translations.
    for i in range(1, 2 ** p + 1):
        t = _node(p, i)
        a, b = cg[t]
        v[t] = H.V[t].T @ X[a:b]
        d[t] = H.D[t] @ X[a:b] if with_diag else 0.0
    for l in range(p - 1, 0, -1):
        for i in range(1, 2 ** l + 1):
            t = _node(l, i)
            v[t] = H.W[t].T @ np.vstack([v[_node(l + 1, 2 * i - 1)], v[_node(l + 1, 2 * i)]])
    # Step 2: core blocks of every sibling pair, stored at the parent.
    for l in range(1, p + 1):
        for i in range(1, 2 ** (l - 1) + 1):
            parent = _node(l - 1, i)
            c1, c2 = _node(l, 2 * i - 1), _node(l, 2 * i)
            w[c1] = H.B12[parent] @ v[c2]
            w[c2] = H.B21[parent] @ v[c1]
    # Step 3: downward pass with the row translations.
    for l in range(1, p):
        for i in range(1, 2 ** l + 1):
            t = _node(l, i)
            c1, c2 = _node(l + 1, 2 * i - 1), _node(l + 1, 2 * i)
            upd = H.R[t] @ w[t]
            k1 = H.ku[c1]
            w[c1] = w[c1] + upd[:k1]
            w[c2] = w[c2] + upd[k1:]
    # Step 4: leaves.
    for i in range(1, 2 ** p + 1):
        t = _node(p, i)
        a, b = rg[t]
        Y[a:b] = H.U[t] @ w[t] + d[t]
    return Y[:, 0] if vec else Y
