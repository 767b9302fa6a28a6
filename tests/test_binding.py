"""Host-side checks of the Python binding and of the test-side start vector
(no GPU needed): arguments the kernels cannot take are rejected before they
reach the library; the splitmix64 start vector matches the generator's
published outputs; the oracle's power method honours a given start vector."""
import numpy as np
import pytest

from oracle import tree
from oracle.hss import HSS
from oracle.norms import norm2_power
from paper_1909_07909_amd import hss, inputs
from startvec import splitmix_raw, splitmix_start

torch = pytest.importorskip("torch")


def test_splitmix_published_outputs():
    # splitmix64 seeded with 0: its first three outputs (states g, 2g, 3g)
    g = 0x9E3779B97F4A7C15
    idx = np.array([0, g, (2 * g) % 2 ** 64], dtype=np.uint64)
    got = [int(x) for x in splitmix_raw(idx, seed=0)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    v = splitmix_start(1000)
    assert v.min() >= -1.0 and v.max() < 1.0 and abs(v.mean()) < 0.1


def test_power_method_start_vector():
    """Started from the top right singular vector, one power step returns
    sigma_1 exactly (to rounding)."""
    g = inputs.synthetic_hss(tree.leaf_offsets(256, 32), 4, seed=1)
    H = HSS.from_packed(g)
    _, s, vt = np.linalg.svd(H.dense())
    assert abs(norm2_power(H, iters=1, x0=vt[0]) - s[0]) <= 1e-12 * s[0]
    # a start vector orthogonal to the top one: the estimate is below sigma_1
    assert norm2_power(H, iters=1, x0=vt[-1]) < s[0] * (1 - 1e-6)


class _Fake(hss.HSSMatrix):
    """An HSSMatrix shell with no device handle: the argument checks run
    before any library call, so they can be exercised without a GPU."""

    def __init__(self, n):
        self.n, self.p, self.h = n, 0, None

    def close(self):
        pass


def test_colmajor_rejects_host_and_dtype():
    n = 8
    with pytest.raises(TypeError):
        hss.colmajor(torch.zeros((n, 2), dtype=torch.float64), n)       # host tensor
    with pytest.raises(TypeError):
        hss.colmajor(np.zeros((n, 2)), n)                                # not a tensor
    A = _Fake(n)
    with pytest.raises(TypeError):
        A.matmul(torch.zeros((2, n), dtype=torch.float64).t())
    with pytest.raises(TypeError):
        A.solve(torch.zeros((2, n), dtype=torch.float32).t())
    with pytest.raises(ValueError):
        hss.batch_solve([A], [])


@pytest.mark.gpu
def test_colmajor_rejects_mixed_dtypes():
    n = 8
    A = _Fake(n)
    X = torch.zeros((2, n), dtype=torch.float64, device="cuda").t()
    Y = torch.zeros((2, n), dtype=torch.float32, device="cuda").t()
    with pytest.raises(TypeError):
        A.matmul(X, Y)
    with pytest.raises(TypeError):
        A.solve(X.float())
    with pytest.raises(ValueError):
        A.matmul(X, torch.zeros((3, n), dtype=torch.float64, device="cuda").t())
    with pytest.raises(TypeError):
        hss.batch_matmul([A, A], [X, X], [X.clone(), Y])


def test_info_layout():
    # HSS_SOLVE_INFO_BYTES(nrhs) = 32 + 8 nrhs: two doubles, four int32
    assert hss.info_bytes(0) == 32 and hss.info_bytes(5) == 72


def test_tune_table_roundtrip():
    """The tuned-choice table as text (no device work): load, read back,
    reject malformed lines without loading anything, reset."""
    hss.tune_reset()
    assert hss.tune_table() == ""
    text = ("128 32 11 0 3 1 4 296.90 349.50 410.00 380.25\n"
            "64 16 5 1 5 0 1 12.00 15.50 8.00 9.25\n")
    hss.tune_load(text)
    rows = sorted(hss.tune_table().strip().split("\n"))
    assert rows == sorted(l.strip() for l in text.strip().split("\n"))
    for bad in ("128 32 11 0 3 1 4 1.0 2.0\n",          # too few fields
                "128 32 11 0 3 2 4 1 2 3 4\n",          # product choice out of range
                "128 32 11 0 3 1 3 1 2 3 4\n",          # columns per wavefront not 0/1/4
                "128 32 11 7 3 1 4 1 2 3 4\n"):         # unknown precision
        with pytest.raises(hss.HSSError):
            hss.tune_load(bad)
    assert len(hss.tune_table().strip().split("\n")) == 2
    hss.tune_reset()
    assert hss.tune_table() == ""


def test_hadamard_and_readback_null_arguments():
    """hss_hadamard and hss_get_generators reject NULL arguments before any
    device work."""
    import ctypes as C
    L = hss.lib()
    h = C.c_void_p()
    assert L.hss_hadamard(None, None, None, None, None) == -5
    assert L.hss_hadamard(None, None, None, None, C.byref(h)) == -1
    assert h.value is None
    assert L.hss_get_generators(None, None, None) == -1
    assert hss.status_str(-2) == "invalid argument"


def test_compress_and_ranks_null_arguments():
    """hss_compress and hss_ranks reject NULL or invalid arguments before any
    device work."""
    import ctypes as C
    L = hss.lib()
    h = C.c_void_p()
    assert L.hss_compress(None, 0.0, None, None, None) == -5
    assert L.hss_compress(None, 0.0, None, None, C.byref(h)) == -1
    assert L.hss_ranks(None, None, None) == -1


def test_construct_dense_arguments():
    """hss_construct_dense rejects invalid arguments before any device work;
    the binding rejects a host tensor."""
    import ctypes as C
    import numpy as np
    import torch
    L = hss.lib()
    h = C.c_void_p()
    fake = C.c_void_p(256)
    lo = np.array([0, 100, 200], dtype=np.int64)
    lp = lo.ctypes.data_as(C.POINTER(C.c_int64))
    assert L.hss_construct_dense(fake, 200, 200, 1, lp, 1e-10, None, None, None) == -9
    assert L.hss_construct_dense(None, 200, 200, 1, lp, 1e-10, None, None, C.byref(h)) == -1
    assert L.hss_construct_dense(fake, 100, 200, 1, lp, 1e-10, None, None, C.byref(h)) == -2
    assert L.hss_construct_dense(fake, 200, 0, 1, lp, 1e-10, None, None, C.byref(h)) == -3
    assert L.hss_construct_dense(fake, 200, 200, -1, lp, 1e-10, None, None, C.byref(h)) == -4
    assert L.hss_construct_dense(fake, 200, 200, 1, None, 1e-10, None, None, C.byref(h)) == -5
    assert L.hss_construct_dense(fake, 201, 201, 1, lp, 1e-10, None, None, C.byref(h)) == -5
    assert L.hss_construct_dense(fake, 200, 200, 1, lp, -1.0, None, None, C.byref(h)) == -6
    assert L.hss_construct_dense(fake, 200, 200, 1, lp, float("nan"), None, None, C.byref(h)) == -6
    big = np.array([0, 129, 200], dtype=np.int64)
    assert L.hss_construct_dense(fake, 200, 200, 1, big.ctypes.data_as(C.POINTER(C.c_int64)),
                                 1e-10, None, None, C.byref(h)) == hss.HSS_EUNSUP
    assert h.value is None
    with pytest.raises(TypeError):
        hss.HSSMatrix.from_dense(torch.zeros(8, 8, dtype=torch.float64), nmin=4)
