"""Seeded synthetic inputs for the HSS matmul / ULV path.

This module only draws random numbers and lays them out in the canonical
packed generator format that ``hss_create`` accepts.  It performs none of the
HSS arithmetic (no products, no factorizations, no tree construction): the
cluster tree (``leaf_off``) and the per-node ranks are arguments.  Both the
FP64 oracle and the GPU path consume what it returns.

Canonical packed format (all blocks column-major, ld = rows, concatenated in
heap order t = 0, 1, ..., 2^(p+1) - 2; node t has children 2t+1, 2t+2):

* ``D``, ``U``, ``V``: leaves only; m_t x m_t, m_t x ku_t, m_t x kv_t.
* ``R``, ``W``: internal nodes except the root;
  (ku_c1 + ku_c2) x ku_t and (kv_c1 + kv_c2) x kv_t (translation operators of
  the nestedness relation, Sec. 2.2).
* ``B12``, ``B21``: every internal node (root included); ku_c1 x kv_c2 and
  ku_c2 x kv_c1 (the core blocks coupling the two children, stored at the
  parent as in the ``hss`` class description of Sec. 2.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Generators:
    n: int
    p: int
    leaf_off: np.ndarray            # int64, 2^p + 1 entries, 0 .. n
    ku: np.ndarray                  # int32, 2^(p+1) - 1 entries (root ignored)
    kv: np.ndarray                  # int32
    D: np.ndarray = field(repr=False)
    U: np.ndarray = field(repr=False)
    V: np.ndarray = field(repr=False)
    R: np.ndarray = field(repr=False)
    W: np.ndarray = field(repr=False)
    B12: np.ndarray = field(repr=False)
    B21: np.ndarray = field(repr=False)

    @property
    def nnodes(self) -> int:
        return 2 ** (self.p + 1) - 1

    def entries(self) -> int:
        return int(sum(a.size for a in (self.D, self.U, self.V, self.R, self.W,
                                        self.B12, self.B21)))


def _is_leaf(t: int, p: int) -> bool:
    return t >= 2 ** p - 1


def _leaf_size(leaf_off: np.ndarray, t: int, p: int) -> int:
    i = t - (2 ** p - 1)
    return int(leaf_off[i + 1] - leaf_off[i])


def haar_orthonormal(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Thin Q of a Gaussian rows x cols matrix with columns sign-fixed so that
    diag(R) > 0 (Haar-distributed orthonormal columns)."""
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return np.asfortranarray(q * s)


class _Packer:
    """Appends column-major blocks in heap order."""

    def __init__(self):
        self.parts = {k: [] for k in ("D", "U", "V", "R", "W", "B12", "B21")}

    def add(self, name: str, block: np.ndarray):
        self.parts[name].append(np.asarray(block, dtype=np.float64).ravel(order="F"))

    def arrays(self):
        out = {}
        for k, v in self.parts.items():
            out[k] = np.concatenate(v) if v else np.zeros(0, dtype=np.float64)
        return out


def uniform_ranks(p: int, k: int) -> tuple[np.ndarray, np.ndarray]:
    nn = 2 ** (p + 1) - 1
    ku = np.full(nn, k, dtype=np.int32)
    kv = np.full(nn, k, dtype=np.int32)
    if p == 0:
        ku[:] = 0
        kv[:] = 0
    else:
        ku[0] = 0
        kv[0] = 0
    return ku, kv


def synthetic_hss(leaf_off, k: int, seed, diag_shift: float | None = None) -> Generators:
    """The synthetic family of the small-parity / headline / batching
    workloads: U_i, V_i Haar-orthonormal (m_i x k); R_t, W_t Haar-orthonormal
    2k x k; B = P diag(sigma) Q^T with sigma_j = 0.5 * 10^(-j/4), P, Q Haar
    k x k; D_i = s*I + G/sqrt(m_i) with s = m_i unless ``diag_shift`` is given.

    Draw order: walk t = 0 .. 2^(p+1)-2; internal non-root: R then W;
    internal: P12, Q12, P21, Q21; leaf: U, V, D.
    ``seed`` may be an int or a numpy SeedSequence."""
    leaf_off = np.asarray(leaf_off, dtype=np.int64)
    nleaf = leaf_off.size - 1
    p = int(round(np.log2(nleaf)))
    assert 2 ** p == nleaf
    n = int(leaf_off[-1])
    ku, kv = uniform_ranks(p, k)
    rng = np.random.default_rng(seed)
    sig = 0.5 * 10.0 ** (-np.arange(k) / 4.0)
    pk = _Packer()
    for t in range(2 ** (p + 1) - 1):
        if _is_leaf(t, p):
            m = _leaf_size(leaf_off, t, p)
            if p > 0:
                pk.add("U", haar_orthonormal(rng, m, k))
                pk.add("V", haar_orthonormal(rng, m, k))
            s = float(m) if diag_shift is None else float(diag_shift)
            pk.add("D", s * np.eye(m) + rng.standard_normal((m, m)) / np.sqrt(m))
        else:
            if t != 0:
                pk.add("R", haar_orthonormal(rng, 2 * k, k))
                pk.add("W", haar_orthonormal(rng, 2 * k, k))
            p12 = haar_orthonormal(rng, k, k)
            q12 = haar_orthonormal(rng, k, k)
            p21 = haar_orthonormal(rng, k, k)
            q21 = haar_orthonormal(rng, k, k)
            pk.add("B12", (p12 * sig) @ q12.T)
            pk.add("B21", (p21 * sig) @ q21.T)
    a = pk.arrays()
    return Generators(n=n, p=p, leaf_off=leaf_off, ku=ku, kv=kv, **a)


def ragged_ranks(p: int, seed, lo: int = 4, hi: int = 16, max_leaf_rank: int | None = None):
    """Per-node ranks (ku, kv) drawn independently, uniform in [lo, hi] at the
    leaves and capped at internal nodes by what the children provide
    (ku_t <= ku_c1 + ku_c2, likewise kv), so that every translation operator
    has at least as many rows as columns.  Root entries are 0."""
    nn = 2 ** (p + 1) - 1
    rng = np.random.default_rng(seed)
    ku = np.zeros(nn, dtype=np.int32)
    kv = np.zeros(nn, dtype=np.int32)
    if p == 0:
        return ku, kv
    cap = hi if max_leaf_rank is None else min(hi, max_leaf_rank)
    for t in range(nn - 1, 0, -1):
        a = int(rng.integers(lo, hi + 1))
        b = int(rng.integers(lo, hi + 1))
        if _is_leaf(t, p):
            ku[t], kv[t] = min(a, cap), min(b, cap)
        else:
            ku[t] = min(a, ku[2 * t + 1] + ku[2 * t + 2])
            kv[t] = min(b, kv[2 * t + 1] + kv[2 * t + 2])
    return ku, kv


def synthetic_hss_ranked(leaf_off, ku, kv, seed) -> Generators:
    """The synthetic family with per-node ranks: U_i (m_i x ku_i), V_i
    (m_i x kv_i), R_t ((ku_c1 + ku_c2) x ku_t), W_t ((kv_c1 + kv_c2) x kv_t)
    Haar-orthonormal; B12_t = P diag(sigma) Q^T of shape ku_c1 x kv_c2 (B21
    ku_c2 x kv_c1) with sigma_j = 0.5 * 10^(-j/4) over min(rows, cols);
    D_i = m_i I + G/sqrt(m_i).  Same draw order as ``synthetic_hss``."""
    leaf_off = np.asarray(leaf_off, dtype=np.int64)
    nleaf = leaf_off.size - 1
    p = int(round(np.log2(nleaf)))
    assert 2 ** p == nleaf
    n = int(leaf_off[-1])
    ku = np.asarray(ku, dtype=np.int32).copy()
    kv = np.asarray(kv, dtype=np.int32).copy()
    ku[0] = kv[0] = 0
    rng = np.random.default_rng(seed)

    def core(rows, cols):
        q = min(rows, cols)
        sig = 0.5 * 10.0 ** (-np.arange(q) / 4.0)
        P = haar_orthonormal(rng, rows, q)
        Q = haar_orthonormal(rng, cols, q)
        return (P * sig) @ Q.T

    pk = _Packer()
    for t in range(2 ** (p + 1) - 1):
        if _is_leaf(t, p):
            m = _leaf_size(leaf_off, t, p)
            if p > 0:
                pk.add("U", haar_orthonormal(rng, m, int(ku[t])))
                pk.add("V", haar_orthonormal(rng, m, int(kv[t])))
            pk.add("D", m * np.eye(m) + rng.standard_normal((m, m)) / np.sqrt(m))
        else:
            c1, c2 = 2 * t + 1, 2 * t + 2
            if t != 0:
                pk.add("R", haar_orthonormal(rng, int(ku[c1] + ku[c2]), int(ku[t])))
                pk.add("W", haar_orthonormal(rng, int(kv[c1] + kv[c2]), int(kv[t])))
            pk.add("B12", core(int(ku[c1]), int(kv[c2])))
            pk.add("B21", core(int(ku[c2]), int(kv[c1])))
    a = pk.arrays()
    return Generators(n=n, p=p, leaf_off=leaf_off, ku=ku, kv=kv, **a)


def rhs(n: int, r: int, seed) -> np.ndarray:
    """n x r standard normal block, Fortran order."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, r)))


# ----------------------------------------------------------------------------
# Structured families whose dense matrix has a closed form (tests compute the
# closed form themselves; here only the generators are laid out).
# ----------------------------------------------------------------------------

def diag_plus_lowrank(leaf_off, k: int, seed) -> tuple[Generators, dict]:
    """Generators of A = diag(d) + U V^T (the 'low-rank' family plus a
    diagonal): leaf bases are the rows of global U, V; every R, W = [I; I];
    every B12 = B21 = I; D_i = diag(d_i) + U_i V_i^T.  Returns the generators
    and the raw factors (d, U, V) for the closed-form checks."""
    leaf_off = np.asarray(leaf_off, dtype=np.int64)
    nleaf = leaf_off.size - 1
    p = int(round(np.log2(nleaf)))
    n = int(leaf_off[-1])
    rng = np.random.default_rng(seed)
    d = 4.0 + rng.uniform(0.0, 1.0, n)
    Ug = rng.standard_normal((n, k)) / np.sqrt(n)
    Vg = rng.standard_normal((n, k)) / np.sqrt(n)
    ku, kv = uniform_ranks(p, k)
    pk = _Packer()
    eye2 = np.vstack([np.eye(k), np.eye(k)])
    for t in range(2 ** (p + 1) - 1):
        if _is_leaf(t, p):
            i = t - (2 ** p - 1)
            a, b = int(leaf_off[i]), int(leaf_off[i + 1])
            Ui, Vi = Ug[a:b], Vg[a:b]
            if p > 0:
                pk.add("U", Ui)
                pk.add("V", Vi)
            pk.add("D", np.diag(d[a:b]) + Ui @ Vi.T)
        else:
            if t != 0:
                pk.add("R", eye2)
                pk.add("W", eye2)
            pk.add("B12", np.eye(k))
            pk.add("B21", np.eye(k))
    a = pk.arrays()
    g = Generators(n=n, p=p, leaf_off=leaf_off, ku=ku, kv=kv, **a)
    return g, {"d": d, "U": Ug, "V": Vg}


def tridiagonal(leaf_off, seed) -> tuple[Generators, dict]:
    """Exact rank-2 HSS generators of a tridiagonal matrix (the 'banded'
    family with one sub- and one super-diagonal).  Leaf bases are
    [e_first, e_last]; R_t = W_t select (first of c1, last of c2);
    B12_t = [[0, 0], [a, 0]] couples the last row of c1 with the first column
    of c2 (superdiagonal entry a); B21_t = [[0, b], [0, 0]] couples the first
    row of c2 with the last column of c1 (subdiagonal entry b).  Returns the
    generators and the three diagonals (lower, main, upper)."""
    leaf_off = np.asarray(leaf_off, dtype=np.int64)
    nleaf = leaf_off.size - 1
    p = int(round(np.log2(nleaf)))
    n = int(leaf_off[-1])
    rng = np.random.default_rng(seed)
    main = 4.0 + rng.uniform(0.0, 1.0, n)
    upper = rng.uniform(-1.0, 1.0, n - 1)
    lower = rng.uniform(-1.0, 1.0, n - 1)
    ku, kv = uniform_ranks(p, 2)
    pk = _Packer()
    sel = np.zeros((4, 2))
    sel[0, 0] = 1.0   # first row of c1 -> first of parent
    sel[3, 1] = 1.0   # last row of c2  -> last of parent
    for t in range(2 ** (p + 1) - 1):
        if _is_leaf(t, p):
            i = t - (2 ** p - 1)
            a, b = int(leaf_off[i]), int(leaf_off[i + 1])
            m = b - a
            E = np.zeros((m, 2))
            E[0, 0] = 1.0
            E[m - 1, 1] = 1.0
            if p > 0:
                pk.add("U", E)
                pk.add("V", E)
            Dm = np.diag(main[a:b])
            if m > 1:
                Dm += np.diag(upper[a:b - 1], 1) + np.diag(lower[a:b - 1], -1)
            pk.add("D", Dm)
        else:
            if t != 0:
                pk.add("R", sel)
                pk.add("W", sel)
            # rightmost leaf of the left child subtree of t
            c = 2 * t + 1
            while not _is_leaf(c, p):
                c = 2 * c + 2
            s = int(leaf_off[c - (2 ** p - 1) + 1]) - 1   # last row of c1
            B12 = np.zeros((2, 2))
            B12[1, 0] = upper[s]
            B21 = np.zeros((2, 2))
            B21[0, 1] = lower[s]
            pk.add("B12", B12)
            pk.add("B21", B21)
    a = pk.arrays()
    g = Generators(n=n, p=p, leaf_off=leaf_off, ku=ku, kv=kv, **a)
    return g, {"lower": lower, "main": main, "upper": upper}


def scaled_identity(leaf_off, k: int, c: float = 1.0) -> Generators:
    """c * I with rank-k bases present but all core blocks zero."""
    return _block_diag_family(leaf_off, k, seed=0, diag=lambda m, rng: c * np.eye(m),
                              zero_core=True)


def block_diagonal(leaf_off, k: int, seed) -> Generators:
    """All core blocks B = 0: A = blkdiag(D_i) with random orthonormal bases."""
    return _block_diag_family(
        leaf_off, k, seed,
        diag=lambda m, rng: m * np.eye(m) + rng.standard_normal((m, m)) / np.sqrt(m),
        zero_core=True)


def _block_diag_family(leaf_off, k, seed, diag, zero_core):
    leaf_off = np.asarray(leaf_off, dtype=np.int64)
    nleaf = leaf_off.size - 1
    p = int(round(np.log2(nleaf)))
    n = int(leaf_off[-1])
    rng = np.random.default_rng(seed)
    ku, kv = uniform_ranks(p, k)
    pk = _Packer()
    for t in range(2 ** (p + 1) - 1):
        if _is_leaf(t, p):
            m = _leaf_size(leaf_off, t, p)
            if p > 0:
                pk.add("U", haar_orthonormal(rng, m, k))
                pk.add("V", haar_orthonormal(rng, m, k))
            pk.add("D", diag(m, rng))
        else:
            if t != 0:
                pk.add("R", haar_orthonormal(rng, 2 * k, k))
                pk.add("W", haar_orthonormal(rng, 2 * k, k))
            pk.add("B12", np.zeros((k, k)))
            pk.add("B21", np.zeros((k, k)))
    a = pk.arrays()
    return Generators(n=n, p=p, leaf_off=leaf_off, ku=ku, kv=kv, **a)


# ----------------------------------------------------------------------------
# Dense inputs of the dense-to-HSS constructor (column-major n x n arrays).
# ----------------------------------------------------------------------------

def cauchy_kernel_dense(n: int, seed: int = 1, width: float = 0.05,
                        shift: float = 1e-2, skew: float = 0.0) -> np.ndarray:
    """The Cauchy-like kernel matrix of the ragged-rank workload: points x_i
    sorted uniform on [0, 1], A_ij = 1 / (1 + ((x_i - x_j) / width)^2) plus
    shift on the diagonal (symmetric positive definite, numerically low-rank
    off-diagonal blocks).  skew != 0 multiplies entry (i, j) by
    1 + skew * tanh((x_i - x_j) / (2 width)): still smooth off the diagonal,
    no longer symmetric."""
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0.0, 1.0, n))
    d = (x[:, None] - x[None, :]) / width
    A = 1.0 / (1.0 + d * d)
    if skew != 0.0:
        A *= 1.0 + skew * np.tanh(0.5 * d)
    A[np.diag_indices_from(A)] += shift
    return np.asfortranarray(A)


def banded_dense(n: int, bl: int, bu: int, seed) -> np.ndarray:
    """Standard normal entries on the band -bl <= j - i <= bu (diagonal
    shifted by bl + bu + 2), zeros elsewhere."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    i, j = np.indices((n, n))
    A[(j - i > bu) | (i - j > bl)] = 0.0
    A[np.diag_indices_from(A)] += bl + bu + 2.0
    return np.asfortranarray(A)
