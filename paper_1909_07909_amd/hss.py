"""Python binding of libhss.so (include/hss.h): argument marshalling only.

Every step of the HSS product and of the ULV factorization / solve runs in
the library's HIP kernels.  PyTorch provides device memory and the stream;
matrices are passed as column-major views: an n x r block is a tensor of
shape (n, r) with strides (1, ld).  If the library is missing this module
raises instead of falling back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhss.so")

(HSS_OK, HSS_ENOMEM, HSS_EHIP, HSS_ESTATE, HSS_ESINGULAR, HSS_ENOCONV, HSS_EUNSUP,
 HSS_ESCRATCH) = range(8)
OP_N, OP_T = 0, 1
F64, F32 = 0, 1

# Every symbol include/hss.h declares.
EXPORTS = (
    "hss_create", "hss_destroy", "hss_matmul", "hss_ulv_factor", "hss_ulv_solve", "hss_query",
    "hss_plan_depth", "hss_plan_leaf_offsets", "hss_plan_node_ranges", "hss_batch_matmul",
    "hss_batch_ulv_factor", "hss_batch_ulv_solve", "hss_status_str", "hss_timing_enable",
    "hss_timing_report", "hss_matmul_noalloc", "hss_matmul_noalloc_max_rhs", "hss_autotune",
    "hss_tune_table", "hss_tune_load", "hss_tune_reset", "hss_hadamard", "hss_get_generators",
    "hss_compress", "hss_ranks", "hss_ulv_factor_solve", "hss_construct_dense",
)

Q_N, Q_P, Q_RESIDENT_BYTES, Q_NORM2, Q_GEN_ENTRIES, Q_FACTOR_ENTRIES = range(6)


class TreeDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("p", C.c_int32), ("reserved", C.c_int32),
                ("leaf_off", C.POINTER(C.c_int64)), ("ku", C.POINTER(C.c_int32)),
                ("kv", C.POINTER(C.c_int32))]


class GenHost(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_double)) for k in ("D", "U", "V", "R", "W", "B12", "B21")]


class GenOut(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_double)) for k in ("D", "U", "V", "R", "W", "B12", "B21")]


class Alloc(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("ctx", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("max_refine", C.c_int32), ("tol", C.c_double),
                ("want_eta", C.c_int32), ("reserved", C.c_int32)]


class SolveInfo(C.Structure):
    """Header of the solve report (followed by ncols doubles of eta_j)."""
    _fields_ = [("eta_max", C.c_double), ("norm2", C.c_double), ("iters", C.c_int32),
                ("status", C.c_int32), ("singular_node", C.c_int32), ("ncols", C.c_int32)]


def info_bytes(nrhs: int) -> int:
    """HSS_SOLVE_INFO_BYTES(nrhs)."""
    return C.sizeof(SolveInfo) + 8 * int(nrhs)


class HSSError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: status {code} ({status_str(code)})")


_lib = None


def lib() -> C.CDLL:
    """Load libhss.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1909_07909_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.hss_create.argtypes = [C.POINTER(TreeDesc), C.POINTER(GenHost), C.POINTER(Alloc), vp,
                             C.POINTER(vp)]
    L.hss_destroy.argtypes = [vp]
    L.hss_hadamard.argtypes = [vp, vp, C.POINTER(Alloc), vp, C.POINTER(vp)]
    L.hss_get_generators.argtypes = [vp, C.POINTER(GenOut), vp]
    L.hss_compress.argtypes = [vp, C.c_double, C.POINTER(Alloc), vp, C.POINTER(vp)]
    L.hss_ranks.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.hss_construct_dense.argtypes = [vp, i64, i64, i32, C.POINTER(C.c_int64), C.c_double,
                                      C.POINTER(Alloc), vp, C.POINTER(vp)]
    L.hss_matmul.argtypes = [vp, i32, i32, i64, vp, i64, vp, i64, vp]
    L.hss_matmul_noalloc.argtypes = [vp, i32, i32, i64, vp, i64, vp, i64, vp]
    L.hss_matmul_noalloc_max_rhs.argtypes = [vp, i32]
    L.hss_ulv_factor.argtypes = [vp, i32, vp]
    L.hss_ulv_solve.argtypes = [vp, i64, vp, i64, C.POINTER(SolveOpts), vp, vp]
    L.hss_ulv_factor_solve.argtypes = [vp, i64, vp, i64, C.POINTER(SolveOpts), vp, vp]
    L.hss_query.argtypes = [vp, i32, vp, vp]
    L.hss_plan_depth.argtypes = [i64, i64]
    L.hss_plan_leaf_offsets.argtypes = [i64, i64, C.POINTER(C.c_int64), i64]
    L.hss_plan_node_ranges.argtypes = [C.POINTER(TreeDesc), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64)]
    L.hss_batch_matmul.argtypes = [C.POINTER(vp), i32, i32, i32, C.POINTER(C.c_int64),
                                   C.POINTER(vp), C.POINTER(C.c_int64), C.POINTER(vp),
                                   C.POINTER(C.c_int64), vp]
    L.hss_batch_ulv_factor.argtypes = [C.POINTER(vp), i32, i32, vp]
    L.hss_batch_ulv_solve.argtypes = [C.POINTER(vp), i32, C.POINTER(C.c_int64), C.POINTER(vp),
                                      C.POINTER(C.c_int64), C.POINTER(SolveOpts),
                                      C.POINTER(vp), vp]
    L.hss_autotune.argtypes = [vp, i64, i32, vp, C.c_char_p, i64]
    L.hss_tune_table.argtypes = [C.c_char_p, i64]
    L.hss_tune_load.argtypes = [C.c_char_p]
    L.hss_tune_reset.argtypes = []
    L.hss_timing_enable.argtypes = [i32]
    L.hss_timing_report.argtypes = [C.c_char_p, i64, i32]
    L.hss_status_str.argtypes = [i32]
    L.hss_status_str.restype = C.c_char_p
    for name in EXPORTS:
        f = getattr(L, name)
        if name != "hss_status_str" and f.restype is not C.c_char_p:
            f.restype = C.c_int32
    L.hss_matmul_noalloc_max_rhs.restype = C.c_int64
    _lib = L
    return L


def status_str(code: int) -> str:
    return lib().hss_status_str(code).decode()


def _check(code, where):
    if code != HSS_OK:
        raise HSSError(code, where)


def plan_depth(n: int, nmin: int) -> int:
    return int(lib().hss_plan_depth(n, nmin))


def plan_leaf_offsets(n: int, nmin: int) -> np.ndarray:
    p = plan_depth(n, nmin)
    out = np.zeros(2 ** p + 1, dtype=np.int64)
    _check(lib().hss_plan_leaf_offsets(n, nmin, out.ctypes.data_as(C.POINTER(C.c_int64)),
                                       out.size), "hss_plan_leaf_offsets")
    return out


def _tree(n, p, leaf_off, ku, kv):
    lo = np.ascontiguousarray(leaf_off, dtype=np.int64)
    ku = np.ascontiguousarray(ku, dtype=np.int32)
    kv = np.ascontiguousarray(kv, dtype=np.int32)
    td = TreeDesc(n, p, 0, lo.ctypes.data_as(C.POINTER(C.c_int64)),
                  ku.ctypes.data_as(C.POINTER(C.c_int32)), kv.ctypes.data_as(C.POINTER(C.c_int32)))
    return td, (lo, ku, kv)


def plan_node_ranges(n, p, leaf_off, ku, kv):
    td, keep = _tree(n, p, leaf_off, ku, kv)
    nn = 2 ** (p + 1) - 1
    start = np.zeros(nn, dtype=np.int64)
    size = np.zeros(nn, dtype=np.int64)
    _check(lib().hss_plan_node_ranges(C.byref(td), start.ctypes.data_as(C.POINTER(C.c_int64)),
                                      size.ctypes.data_as(C.POINTER(C.c_int64))),
           "hss_plan_node_ranges")
    return start, size


def tune_table() -> str:
    """The autotuned launch choices recorded so far (text, one line per shape class)."""
    buf = C.create_string_buffer(1 << 16)
    _check(lib().hss_tune_table(buf, len(buf)), "hss_tune_table")
    return buf.value.decode()


def tune_load(text: str):
    """Load choices written by tune_table()."""
    _check(lib().hss_tune_load(text.encode()), "hss_tune_load")


def tune_reset():
    _check(lib().hss_tune_reset(), "hss_tune_reset")


def timing_enable(on: bool):
    lib().hss_timing_enable(1 if on else 0)


def timing_report(reset: bool = True):
    """Per-kernel event timings since the last reset: list of dicts."""
    import json
    buf = C.create_string_buffer(1 << 16)
    _check(lib().hss_timing_report(buf, len(buf), 1 if reset else 0), "hss_timing_report")
    return json.loads(buf.value.decode())


def _stream(stream):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(stream)


def colmajor(t, n, dtypes=None):
    """(ptr, ld) of a column-major (n, r) CUDA tensor view (strides (1, ld)).

    dtypes: the accepted torch dtypes (None: float64 and float32).  Raises
    TypeError for a host tensor or another dtype and ValueError for a shape
    or layout the kernels cannot take, before anything reaches the library."""
    import torch
    if dtypes is None:
        dtypes = (torch.float64, torch.float32)
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise TypeError("tensor must be in GPU memory (device='cuda')")
    if t.dtype not in dtypes:
        raise TypeError(f"tensor dtype {t.dtype} not accepted here (expected one of {dtypes})")
    if t.dim() != 2 or t.shape[0] != n:
        raise ValueError(f"expected an ({n}, r) tensor, got {tuple(t.shape)}")
    # (the row stride of a one-row tensor is immaterial)
    if n > 1 and t.shape[1] > 1 and t.stride(0) != 1:
        raise ValueError("tensor must be column-major: strides (1, ld)")
    if n > 1 and t.shape[1] == 1 and t.stride(0) != 1:
        raise ValueError("tensor must have unit row stride")
    ld = t.stride(1) if t.shape[1] > 1 else max(t.stride(1), n)
    return C.c_void_p(t.data_ptr()), ld


def empty_colmajor(n, r, dtype, device="cuda"):
    import torch
    return torch.empty((r, n), dtype=dtype, device=device).t()


# Device allocator hooks backed by PyTorch's caching allocator (the memory of
# a handle then counts in torch.cuda.memory_allocated).  Module-level, so the
# callbacks outlive every handle that uses them.
def _torch_alloc(nbytes, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes))
    except RuntimeError:
        return None


def _torch_free(ptr, ctx):
    import torch
    torch.cuda.caching_allocator_delete(ptr)


TORCH_ALLOC = Alloc(Alloc._fields_[0][1](_torch_alloc), Alloc._fields_[1][1](_torch_free), None)


class SolveReport:
    """The solve report the device writes (pinned host memory).  Read it with
    result() once the stream has reached the end of the solve."""

    def __init__(self, nrhs):
        import torch
        self.nrhs = int(nrhs)
        self.buf = torch.zeros(info_bytes(nrhs), dtype=torch.uint8, pin_memory=True)

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())

    def result(self):
        raw = self.buf.numpy()
        hdr = SolveInfo.from_buffer_copy(raw[:C.sizeof(SolveInfo)].tobytes())
        eta = np.frombuffer(raw[C.sizeof(SolveInfo):].tobytes(), dtype=np.float64)
        return {"status": int(hdr.status), "eta": eta[:self.nrhs].copy(),
                "eta_max": float(hdr.eta_max), "iters": int(hdr.iters), "norm2": float(hdr.norm2),
                "singular_node": int(hdr.singular_node), "ncols": int(hdr.ncols)}


def _sync(stream):
    import torch
    if stream is None:
        torch.cuda.current_stream().synchronize()
    elif hasattr(stream, "synchronize"):
        stream.synchronize()
    else:
        torch.cuda.synchronize()


_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    # handles whose memory came from PyTorch's allocator are released before
    # the interpreter (and the allocator's Python entry points) shut down
    for m in list(_LIVE):
        try:
            m.close()
        except Exception:
            pass


class _Gens:
    """Plain holder of a read-back tree and generator arrays."""


class HSSMatrix:
    """Device-resident HSS matrix created from generators in the canonical
    packed layout (attributes n, p, leaf_off, ku, kv, D, U, V, R, W, B12, B21).

    alloc: "torch" (default) allocates the handle's device memory from
    PyTorch's caching allocator, None uses hipMalloc, or an Alloc structure."""

    def __init__(self, g, stream=None, alloc="torch"):
        L = lib()
        td, self._keep = _tree(g.n, g.p, g.leaf_off, g.ku, g.kv)
        arrs = [np.ascontiguousarray(getattr(g, k), dtype=np.float64)
                for k in ("D", "U", "V", "R", "W", "B12", "B21")]
        gh = GenHost(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs])
        if isinstance(alloc, str):
            if alloc != "torch":
                raise ValueError(f"unknown allocator {alloc!r}")
            alloc = TORCH_ALLOC
        self._alloc = alloc
        h = C.c_void_p()
        code = L.hss_create(C.byref(td), C.byref(gh), C.byref(alloc) if alloc else None,
                            _stream(stream), C.byref(h))
        _check(code, "hss_create")
        self._adopt(h, g.n, g.p, g.leaf_off, g.ku, g.kv)

    def _adopt(self, h, n, p, leaf_off, ku, kv):
        self.h = h
        self.n = int(n)
        self.p = int(p)
        self.leaf_off = np.asarray(leaf_off, dtype=np.int64).copy()
        self.ku = np.asarray(ku, dtype=np.int32).copy()
        self.kv = np.asarray(kv, dtype=np.int32).copy()
        self.ku[0] = self.kv[0] = 0
        _LIVE.add(self)

    def hadamard(self, other, stream=None, alloc="torch"):
        """The elementwise product self o other (same tree) as a new
        HSSMatrix, formed on the device by hss_hadamard."""
        if isinstance(alloc, str):
            if alloc != "torch":
                raise ValueError(f"unknown allocator {alloc!r}")
            alloc = TORCH_ALLOC
        h = C.c_void_p()
        code = lib().hss_hadamard(self.h, other.h, C.byref(alloc) if alloc else None,
                                  _stream(stream), C.byref(h))
        _check(code, "hss_hadamard")
        out = HSSMatrix.__new__(HSSMatrix)
        out._alloc = alloc
        out._keep = None
        out._adopt(h, self.n, self.p, self.leaf_off, self.ku.astype(np.int64) * other.ku,
                   self.kv.astype(np.int64) * other.kv)
        return out

    @classmethod
    def from_dense(cls, A, leaf_off=None, nmin=None, eps=1e-12, stream=None, alloc="torch"):
        """The HSS approximation of a dense n x n float64 CUDA matrix A
        (column-major view, e.g. M.t() of a contiguous tensor M = A^T) by
        hss_construct_dense: truncation tolerance eps relative to each
        block's largest singular value; the tree from leaf_off or from the
        default split with leaves of at most nmin rows."""
        import torch
        n = int(A.shape[0])
        if A.dim() != 2 or A.shape[1] != n:
            raise ValueError(f"A must be square, got {tuple(A.shape)}")
        ap, lda = colmajor(A, n, (torch.float64,))
        if (leaf_off is None) == (nmin is None):
            raise ValueError("give exactly one of leaf_off and nmin")
        lo = plan_leaf_offsets(n, nmin) if leaf_off is None else np.asarray(leaf_off, dtype=np.int64)
        lo = np.ascontiguousarray(lo, dtype=np.int64)
        p = int(round(np.log2(lo.size - 1)))
        if 2 ** p + 1 != lo.size:
            raise ValueError("leaf_off must have 2^p + 1 entries")
        if isinstance(alloc, str):
            if alloc != "torch":
                raise ValueError(f"unknown allocator {alloc!r}")
            alloc = TORCH_ALLOC
        h = C.c_void_p()
        code = lib().hss_construct_dense(ap, lda, n, p, lo.ctypes.data_as(C.POINTER(C.c_int64)),
                                         float(eps), C.byref(alloc) if alloc else None,
                                         _stream(stream), C.byref(h))
        _check(code, "hss_construct_dense")
        nn = 2 ** (p + 1) - 1
        ku = np.zeros(nn, dtype=np.int32)
        kv = np.zeros(nn, dtype=np.int32)
        _check(lib().hss_ranks(h, ku.ctypes.data_as(C.POINTER(C.c_int32)),
                               kv.ctypes.data_as(C.POINTER(C.c_int32))), "hss_ranks")
        out = cls.__new__(cls)
        out._alloc = alloc
        out._keep = None
        out._adopt(h, n, p, lo, ku, kv)
        return out

    def compress(self, tau=None, rel=None, stream=None, alloc="torch"):
        """Recompression (hss_compress) with absolute tolerance tau, or
        tau = rel * ||A||_2 (the handle's estimate); a new HSSMatrix."""
        if (tau is None) == (rel is None):
            raise ValueError("give exactly one of tau and rel")
        if tau is None:
            tau = float(rel) * self.norm2()
        if isinstance(alloc, str):
            if alloc != "torch":
                raise ValueError(f"unknown allocator {alloc!r}")
            alloc = TORCH_ALLOC
        h = C.c_void_p()
        code = lib().hss_compress(self.h, float(tau), C.byref(alloc) if alloc else None,
                                  _stream(stream), C.byref(h))
        _check(code, "hss_compress")
        nn = 2 ** (self.p + 1) - 1
        ku = np.zeros(nn, dtype=np.int32)
        kv = np.zeros(nn, dtype=np.int32)
        _check(lib().hss_ranks(h, ku.ctypes.data_as(C.POINTER(C.c_int32)),
                               kv.ctypes.data_as(C.POINTER(C.c_int32))), "hss_ranks")
        out = HSSMatrix.__new__(HSSMatrix)
        out._alloc = alloc
        out._keep = None
        out._adopt(h, self.n, self.p, self.leaf_off, ku, kv)
        return out

    def packed_sizes(self):
        """Entry counts of the canonical packed arrays D, U, V, R, W, B12, B21."""
        p, ku, kv, lo = self.p, self.ku, self.kv, self.leaf_off
        sz = dict(D=0, U=0, V=0, R=0, W=0, B12=0, B21=0)
        for t in range(2 ** (p + 1) - 1):
            if t >= 2 ** p - 1:
                m = int(lo[t - (2 ** p - 1) + 1] - lo[t - (2 ** p - 1)])
                sz["D"] += m * m
                if p > 0:
                    sz["U"] += m * int(ku[t])
                    sz["V"] += m * int(kv[t])
            else:
                c1, c2 = 2 * t + 1, 2 * t + 2
                if t != 0:
                    sz["R"] += int(ku[c1] + ku[c2]) * int(ku[t])
                    sz["W"] += int(kv[c1] + kv[c2]) * int(kv[t])
                sz["B12"] += int(ku[c1]) * int(kv[c2])
                sz["B21"] += int(ku[c2]) * int(kv[c1])
        return sz

    def generators(self, stream=None):
        """The FP64 generators read back (hss_get_generators) as an object
        with n, p, leaf_off, ku, kv and the packed arrays D .. B21."""
        sz = self.packed_sizes()
        arrs = {k: np.zeros(v, dtype=np.float64) for k, v in sz.items()}
        go = GenOut(*[arrs[k].ctypes.data_as(C.POINTER(C.c_double))
                      for k in ("D", "U", "V", "R", "W", "B12", "B21")])
        _check(lib().hss_get_generators(self.h, C.byref(go), _stream(stream)),
               "hss_get_generators")
        g = _Gens()
        g.n, g.p, g.leaf_off, g.ku, g.kv = self.n, self.p, self.leaf_off, self.ku, self.kv
        for k, v in arrs.items():
            setattr(g, k, v)
        return g

    def close(self):
        if getattr(self, "h", None):
            lib().hss_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matmul(self, X, Y=None, op=OP_N, stream=None):
        """Y = op(A) X for a column-major (n, r) CUDA tensor (float64 or float32);
        Y, if given, must have X's dtype."""
        import torch
        xp, ldx = colmajor(X, self.n)
        prec = F64 if X.dtype == torch.float64 else F32
        r = X.shape[1]
        if Y is None:
            Y = empty_colmajor(self.n, r, X.dtype, X.device)
        yp, ldy = colmajor(Y, self.n, (X.dtype,))
        if Y.shape[1] != r:
            raise ValueError(f"Y has {Y.shape[1]} columns, X has {r}")
        _check(lib().hss_matmul(self.h, op, prec, r, xp, ldx, yp, ldy, _stream(stream)),
               "hss_matmul")
        return Y

    def matmul_noalloc(self, X, Y, op=OP_N, stream=None):
        """Y = op(A) X through hss_matmul_noalloc (work vectors in the library's
        fixed device scratch; Y must be given).  Raises HSSError with
        HSS_ESCRATCH when the product does not fit that scratch."""
        import torch
        xp, ldx = colmajor(X, self.n)
        yp, ldy = colmajor(Y, self.n, (X.dtype,))
        if Y.shape[1] != X.shape[1]:
            raise ValueError(f"Y has {Y.shape[1]} columns, X has {X.shape[1]}")
        prec = F64 if X.dtype == torch.float64 else F32
        _check(lib().hss_matmul_noalloc(self.h, op, prec, X.shape[1], xp, ldx, yp, ldy,
                                        _stream(stream)), "hss_matmul_noalloc")
        return Y

    def noalloc_max_rhs(self, prec=F64):
        return int(lib().hss_matmul_noalloc_max_rhs(self.h, prec))

    def factor(self, prec=F64, stream=None):
        _check(lib().hss_ulv_factor(self.h, prec, _stream(stream)), "hss_ulv_factor")

    def solve(self, B, prec=F64, tol=0.0, max_refine=10, want_eta=False, stream=None,
              check=True, sync=True, report=None):
        """B <- A^{-1} B in place (column-major float64 CUDA tensor).

        sync=True: waits for the stream and returns a dict with eta (per
        column), eta_max, iters, status, norm2 and singular_node, raising
        HSSError for a status other than HSS_OK when check is set.
        sync=False: returns the SolveReport (read it after the stream has
        reached the end of the solve); nothing waits.  report: a SolveReport
        to write (e.g. one allocated before a graph capture)."""
        import torch
        bp, ldb = colmajor(B, self.n, (torch.float64,))
        r = B.shape[1]
        opts = SolveOpts(prec, max_refine, tol, 1 if want_eta else 0, 0)
        rep = SolveReport(r) if report is None else report
        if rep.nrhs < r:
            raise ValueError(f"report holds {rep.nrhs} columns, the solve has {r}")
        code = lib().hss_ulv_solve(self.h, r, bp, ldb, C.byref(opts), rep.ptr, _stream(stream))
        _check(code, "hss_ulv_solve")
        if not sync:
            return rep
        _sync(stream)
        out = rep.result()
        if check and out["status"] != HSS_OK:
            raise HSSError(out["status"], "hss_ulv_solve")
        return out

    def factor_solve(self, B, prec=F64, tol=0.0, max_refine=10, want_eta=False, stream=None,
                     check=True, sync=True, report=None):
        """Factor with prec, then B <- A^{-1} B in place, in one call
        (hss_ulv_factor_solve; in FP64 the first solve's forward sweep
        overlapped with the factorization); arguments and result as solve().

        sync=True: waits for the stream and returns a dict with eta (per
        column), eta_max, iters, status, norm2 and singular_node, raising
        HSSError for a status other than HSS_OK when check is set.
        sync=False: returns the SolveReport (read it after the stream has
        reached the end of the solve); nothing waits.  report: a SolveReport
        to write (e.g. one allocated before a graph capture)."""
        import torch
        bp, ldb = colmajor(B, self.n, (torch.float64,))
        r = B.shape[1]
        opts = SolveOpts(prec, max_refine, tol, 1 if want_eta else 0, 0)
        rep = SolveReport(r) if report is None else report
        if rep.nrhs < r:
            raise ValueError(f"report holds {rep.nrhs} columns, the solve has {r}")
        code = lib().hss_ulv_factor_solve(self.h, r, bp, ldb, C.byref(opts), rep.ptr,
                                          _stream(stream))
        _check(code, "hss_ulv_factor_solve")
        if not sync:
            return rep
        _sync(stream)
        out = rep.result()
        if check and out["status"] != HSS_OK:
            raise HSSError(out["status"], "hss_ulv_factor_solve")
        return out

    def solve_async(self, B, prec=F64, stream=None):
        """Plain solve without a backward error or report: no synchronization."""
        import torch
        r = B.shape[1]
        bp, ldb = colmajor(B, self.n, (torch.float64,))
        opts = SolveOpts(prec, 0, 0.0, 0, 0)
        _check(lib().hss_ulv_solve(self.h, r, bp, ldb, C.byref(opts), None, _stream(stream)),
               "hss_ulv_solve")

    def autotune(self, nrhs: int, prec=F64, stream=None) -> dict:
        """Time the launch variants for products and solves of nrhs columns
        on this matrix and record the faster for its shape class (see
        hss_autotune); returns the report.  Synchronizes the stream."""
        import json
        if int(nrhs) < 1:
            raise ValueError("nrhs must be >= 1")
        buf = C.create_string_buffer(1024)
        _check(lib().hss_autotune(self.h, int(nrhs), int(prec), _stream(stream), buf, len(buf)),
               "hss_autotune")
        return json.loads(buf.value.decode())

    def query(self, key, stream=None):
        if key in (Q_N, Q_RESIDENT_BYTES, Q_GEN_ENTRIES, Q_FACTOR_ENTRIES):
            v = C.c_int64()
        elif key == Q_P:
            v = C.c_int32()
        else:
            v = C.c_double()
        _check(lib().hss_query(self.h, key, C.byref(v), _stream(stream)), "hss_query")
        return v.value

    def norm2(self, stream=None):
        return self.query(Q_NORM2, stream)


def _ptr_array(items):
    return (C.c_void_p * len(items))(*[C.c_void_p(x) for x in items])


def batch_factor(mats, prec=F64, stream=None):
    hs = _ptr_array([m.h.value for m in mats])
    _check(lib().hss_batch_ulv_factor(hs, len(mats), prec, _stream(stream)),
           "hss_batch_ulv_factor")


def batch_matmul(mats, Xs, Ys, op=OP_N, stream=None):
    import torch
    if not (len(mats) == len(Xs) == len(Ys)):
        raise ValueError("mats, Xs and Ys must have the same length")
    if not mats:
        return
    dt = Xs[0].dtype
    if dt not in (torch.float64, torch.float32):
        raise TypeError("X must be float64 or float32")
    prec = F64 if dt == torch.float64 else F32
    xp, lx, yp, ly = [], [], [], []
    for m, x, y in zip(mats, Xs, Ys):
        a, b = colmajor(x, m.n, (dt,))
        c, d = colmajor(y, m.n, (dt,))
        if y.shape[1] != x.shape[1]:
            raise ValueError("each Y must have its X's column count")
        xp.append(a.value); lx.append(b); yp.append(c.value); ly.append(d)
    hs = _ptr_array([m.h.value for m in mats])
    nr = (C.c_int64 * len(mats))(*[x.shape[1] for x in Xs])
    _check(lib().hss_batch_matmul(hs, len(mats), op, prec, nr, _ptr_array(xp),
                                  (C.c_int64 * len(mats))(*lx), _ptr_array(yp),
                                  (C.c_int64 * len(mats))(*ly), _stream(stream)),
           "hss_batch_matmul")


def batch_solve(mats, Bs, prec=F64, tol=0.0, max_refine=10, want_eta=False, stream=None,
                sync=True, reports=None):
    """B_i <- A_i^{-1} B_i for every instance (one launch per tree level).
    sync=True: waits and returns one report dict per instance; sync=False
    returns the SolveReports.  reports: SolveReports to write (e.g. allocated
    before a graph capture)."""
    import torch
    if len(mats) != len(Bs):
        raise ValueError("mats and Bs must have the same length")
    cnt = len(mats)
    bp, lb = [], []
    for m, b in zip(mats, Bs):
        a, l = colmajor(b, m.n, (torch.float64,))
        bp.append(a.value); lb.append(l)
    hs = _ptr_array([m.h.value for m in mats])
    nr = (C.c_int64 * cnt)(*[b.shape[1] for b in Bs])
    opts = SolveOpts(prec, max_refine, tol, 1 if want_eta else 0, 0)
    reps = [SolveReport(b.shape[1]) for b in Bs] if reports is None else list(reports)
    if len(reps) != cnt or any(r.nrhs < b.shape[1] for r, b in zip(reps, Bs)):
        raise ValueError("one report per instance, each with room for its columns")
    code = lib().hss_batch_ulv_solve(hs, cnt, nr, _ptr_array(bp), (C.c_int64 * cnt)(*lb),
                                     C.byref(opts), _ptr_array([r.ptr.value for r in reps]),
                                     _stream(stream))
    _check(code, "hss_batch_ulv_solve")
    if not sync:
        return reps
    _sync(stream)
    return [r.result() for r in reps]
