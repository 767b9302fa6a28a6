"""||A||_2 estimate and the normwise backward error.

Test infrastructure only (see ``oracle/__init__``).

* Sec. 4.5: before recompressing, the toolbox estimates ||A||_2 by the power
  method on A A^*.  ``norm2_power`` runs the power method on A^T A with the
  oracle's HSS products (A x and A^T y), from a seeded Gaussian start, and
  returns sqrt of the Rayleigh quotient, a lower bound of ||A||_2.
* Sec. 5.1 reports the relative residual ||T x - b||_2 / (||T||_2 ||x||_2 + ||b||_2)
  of its Toeplitz solver (the printed denominator has "v" for b).
  ``backward_error`` evaluates it per column; the solver results of this
  build state it for every right-hand side.

Pins (tests/test_oracle_norms.py): numpy's exact 2-norm of the assembled
matrix, the closed-form spectrum of the (2, -1) tridiagonal matrix, c*I;
eta = 1 for x = 0, and eta for an exactly scaled solution.
"""
from __future__ import annotations

import numpy as np

from .hss import HSS
from .matvec import matvec


def norm2_power(H: HSS, iters: int = 50, seed: int = 12345, x0=None) -> float:
    """sqrt of x^T A^T A x after ``iters`` power steps; x0 (optional) is the
    start vector, else a seeded Gaussian one."""
    if x0 is None:
        x = np.random.default_rng(seed).standard_normal(H.n)
    else:
        x = np.array(x0, dtype=np.float64)
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = matvec(H, x, "N")
        z = matvec(H, y, "T")
        lam = float(np.dot(x, z))          # x^T A^T A x with ||x|| = 1
        nz = np.linalg.norm(z)
        if nz == 0.0:
            return 0.0
        x = z / nz
    return float(np.sqrt(max(lam, 0.0)))


def backward_error(H: HSS, X, B, normA: float) -> np.ndarray:
    """eta_j = ||b_j - A x_j|| / (||A|| ||x_j|| + ||b_j||) for each column."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64).T).T
    B = np.atleast_2d(np.asarray(B, dtype=np.float64).T).T
    Rres = B - matvec(H, X, "N")
    num = np.linalg.norm(Rres, axis=0)
    den = normA * np.linalg.norm(X, axis=0) + np.linalg.norm(B, axis=0)
    return num / den
