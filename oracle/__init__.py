"""FP64 CPU oracle for the HSS matrix x block product and the ULV solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  The product path (the HIP
library and its Python binding) never calls into it, and it shares no code
with that path: it reads the canonical packed generator arrays with its own
unpacker and follows the paper's algorithms in the paper's order.

Modules
-------
tree      cluster tree of Def. 2.1 with the default split rule of Sec. 3.1
hss       unpacked generators (Sec. 2.2), explicit nested bases, dense assembly
matvec    the four-step HSS matrix-vector product (Sec. 4.1, Fig. "mat-vec")
ulv       A^{-1}B by the four steps of Sec. 4.3 (QL / LQ sparsification,
          Woodbury split A~ = A1 A2, recursion on the merged leaves, apply Z)
norms     power method on A^T A for ||A||_2 (Sec. 4.5) and the normwise
          backward error used in Sec. 5.1
hadamard  the Hadamard product of two HSS matrices on one tree (Sec. 4.4):
          elementwise D, transpose Khatri-Rao bases, Kronecker translation
          operators and core blocks
compress  HSS recompression (Sec. 4.5, App. A): proper form by bottom-up
          QR, then top-down truncated SVDs of the core blocks
construct the dense-to-HSS constructor (Sec. 3.2): truncated SVDs of
          the block rows and columns from the leaves up, nested through a
          reduced matrix

Every function is pinned in ``tests/test_oracle_*.py`` against closed forms,
dense LAPACK, brute force or the worked example of Fig. 1 (see each module's
header for the pins).  Parity unpinned: none of the public functions.
"""
