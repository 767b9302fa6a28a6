"""Continuous-batching HSS solve server.

Requests (matrix id, right-hand-side block, target backward error) arrive
while earlier ones run on the GPU.  The factored matrices stay resident in HBM
(a catalogue of HSSMatrix objects, FP32 ULV factors).  Worker threads, one
HIP stream each, repeatedly form a round from the admitted requests:

* admission is by device memory: a request is admitted once the bytes of its
  right-hand sides and refinement buffers fit in the in-flight budget;
* a round takes the admitted requests in arrival order, at most one group per
  matrix and only matrices no other worker is using; requests on the same
  matrix and tolerance class merge into one multi-column block;
* a round runs one batched solve per tolerance class (one launch per tree
  level across all its matrices, FP32 sweeps with FP64 refinement until the
  class tolerance); requests that arrive meanwhile are admitted as memory frees
  and picked up by the next free worker, so rounds overlap on the device.

A catalogue bounds residency: it holds every matrix's generators on the host
and keeps at most a device-memory budget of them resident, created and
FP32-factored when a round first needs them, least recently used idle ones
evicted to make room (a matrix a round is using is never evicted).

Each completed request records its latency (arrival to result: on the
host for host requests, in device memory for device-resident requests) and
the backward error of every column.  The GPU work is all in libhss.so;
this module only schedules.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import hss, inputs


@dataclass
class Request:
    rid: int
    mat: int
    tol: float
    nrhs: int
    t_arrival: float
    B: object = field(repr=False, default=None)   # n x nrhs: numpy (host) or device tensor
    X: object = field(repr=False, default=None)   # result, same kind as B
    eta: np.ndarray = field(repr=False, default=None)
    iters: int = 0
    t_done: float = 0.0
    status: int = 0


def request_bytes(n: int, nrhs: int) -> int:
    """Device bytes a request holds while in flight: its FP64 right-hand side
    block plus the FP64 refinement copies (b0, residual, correction) and the
    FP32 working block."""
    return n * nrhs * (8 * 4 + 4)


def draw_catalogue(count: int, seed: int, n_lo: int = 4096, n_hi: int = 2 ** 20,
                   leaf: int = 128, ranks=(16, 32, 64)):
    """(n, k) of the resident matrices: n log-uniform in [n_lo, n_hi] rounded to
    a multiple of the leaf size, k uniform over ``ranks``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))) / leaf)) * leaf
        n = max(leaf, n)
        out.append((n, int(rng.choice(ranks))))
    return out


def _gen_one(args):
    n, k, seed, leaf = args
    lo = hss.plan_leaf_offsets(n, leaf)
    return inputs.synthetic_hss(lo, k, seed=seed)


def build_catalogue(specs, seed: int, leaf: int = 128, workers: int = 8):
    """Generators of the catalogue (host), drawn in parallel processes."""
    from concurrent.futures import ProcessPoolExecutor
    jobs = [(n, k, seed * 1000 + j, leaf) for j, (n, k) in enumerate(specs)]
    if workers <= 1:
        return [_gen_one(j) for j in jobs]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_gen_one, jobs))


def poisson_requests(rate: float, duration: float, n_mats: int, seed: int,
                     tols=(1e-6, 1e-10), max_rhs: int = 16):
    """Arrival times (exponential gaps at ``rate`` per second), matrix ids,
    tolerance class (equal odds) and block widths U{1..max_rhs}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append(Request(rid=rid, mat=int(rng.integers(n_mats)), tol=float(rng.choice(tols)),
                           nrhs=int(rng.integers(1, max_rhs + 1)), t_arrival=t))
        rid += 1
    return out


def rhs_for(req: Request, n: int) -> np.ndarray:
    return inputs.rhs(n, req.nrhs, 10_000 + req.rid)


def rhs_pools(mats, width: int = 32, seed: int = 77, device: bool = False):
    """One seeded n x width random block per matrix; a request takes a window
    of consecutive columns (so that long runs do not draw fresh normals for
    every request).  device=True: the pools are column-major device tensors
    (requests then carry device views, as from a client on the GPU)."""
    ns = list(mats.n) if isinstance(mats, Catalogue) else [m.n for m in mats]
    pools = [inputs.rhs(n, width, seed + j) for j, n in enumerate(ns)]
    if device:
        import torch
        pools = [torch.from_numpy(np.ascontiguousarray(P.T)).cuda().t() for P in pools]
    return pools


def rhs_from_pool(req: Request, pools) -> np.ndarray:
    P = pools[req.mat]
    s = req.rid % (P.shape[1] - req.nrhs + 1)
    return P[:, s:s + req.nrhs]


class Catalogue:
    """Matrices a server solves with: generators on the host, at most
    ``budget_bytes`` of them resident on the device.  ``acquire(j)`` returns
    matrix j created and FP32-factored (and its work buffers sized for
    ``max_cols`` columns), creating it if it is not resident and first
    evicting least recently used matrices that no round is using until it
    fits; ``release(j)`` ends a round's use.  A matrix that alone exceeds the
    budget is still loaded (the budget is then exceeded by it alone)."""

    def __init__(self, gens, budget_bytes: int, max_cols: int = 64):
        import torch
        self.torch = torch
        self.gens = list(gens)
        self.n = [g.n for g in self.gens]
        self.budget = int(budget_bytes)
        self.max_cols = max_cols
        self.resident = {}            # j -> HSSMatrix
        self.bytes = {}               # j -> resident bytes (measured at load)
        self.last = {}                # j -> use clock
        self.users = {}               # j -> rounds using it
        self.seen = {}                # j -> bytes measured at its last load
        self.clock = 0
        self.hits = self.misses = self.evictions = 0
        self.load_s = 0.0
        self.lock = threading.Lock()

    def __len__(self):
        return len(self.gens)

    def resident_bytes(self) -> int:
        with self.lock:
            return sum(self.bytes.values())

    def is_resident(self, j: int) -> bool:
        with self.lock:
            return j in self.resident

    def expected_bytes(self, j: int) -> int:
        """Device bytes matrix j takes when resident: measured once loaded,
        else estimated from its generators (FP64 + FP32 copies and an FP32
        factor set of about their size)."""
        with self.lock:
            b = self.bytes.get(j)
        if b is None:
            b = self.seen.get(j)
        return int(b) if b else int(16 * self.gens[j].entries())

    def _evict_for_locked(self, need: int):
        while self.resident and sum(self.bytes.values()) + need > self.budget:
            idle = [j for j in self.resident if self.users.get(j, 0) == 0]
            if not idle:
                return
            j = min(idle, key=lambda q: self.last[q])
            self.resident.pop(j).close()
            self.bytes.pop(j)
            self.evictions += 1

    def acquire(self, j: int):
        with self.lock:
            self.clock += 1
            self.last[j] = self.clock
            self.users[j] = self.users.get(j, 0) + 1
            if j in self.resident:
                self.hits += 1
                return self.resident[j]
            self.misses += 1
            # the expected size: a matrix of the same shape loaded before, else
            # the FP64 + FP32 generators and an FP32 factor set of about their size
            est = self.seen.get(j) or int(16 * self.gens[j].entries())
            self._evict_for_locked(est)
        t0 = time.perf_counter()
        try:
            A = hss.HSSMatrix(self.gens[j])
            A.factor(hss.F32)
            A.norm2()
            B = hss.empty_colmajor(A.n, self.max_cols, self.torch.float64)
            B.fill_(1.0)
            A.solve(B, prec=hss.F32, tol=1e-10, max_refine=1, check=False)
            del B
        except Exception:
            with self.lock:
                self.users[j] -= 1
            raise
        with self.lock:
            self.resident[j] = A
            self.bytes[j] = self.seen[j] = int(A.query(hss.Q_RESIDENT_BYTES))
            self.load_s += time.perf_counter() - t0
            self._evict_for_locked(0)
        return A

    def release(self, j: int):
        with self.lock:
            self.users[j] -= 1

    def stats(self) -> dict:
        with self.lock:
            return {"hits": self.hits, "misses": self.misses, "evictions": self.evictions,
                    "resident": len(self.resident), "resident_bytes": sum(self.bytes.values()),
                    "budget_bytes": self.budget, "load_s": round(self.load_s, 3)}


class Server:
    def __init__(self, mats, budget_bytes: int, workers: int = 2, max_mats_per_round: int = 64,
                 max_cols_per_group: int = 64, max_refine: int = 10, max_wait_s: float = 0.05):
        """mats: resident, FP32-factored HSSMatrix objects, or a Catalogue
        (created and evicted as rounds need them; requests on matrices that
        are not resident wait up to max_wait_s for others to share a load)."""
        import torch
        self.torch = torch
        self.mats = mats
        self.cat = mats if isinstance(mats, Catalogue) else None
        self.n = list(mats.n) if self.cat is not None else [m.n for m in mats]
        self.budget = budget_bytes
        self.max_mats = max_mats_per_round
        self.max_cols = max_cols_per_group
        self.max_refine = max_refine
        self.max_wait_s = max_wait_s
        self.pending = deque()        # arrived, waiting for memory
        self.admitted = deque()       # admitted, waiting for a round
        self.inflight_bytes = 0
        self.peak_bytes = 0
        self.busy = set()             # matrices used by a running round
        self.done = []
        self.cv = threading.Condition()
        self.closed = False
        self.nworkers = workers
        self.rounds = 0
        self.round_sizes = []
        self.errors = []
        self.phase_s = {"stage_in": 0.0, "solve": 0.0, "stage_out": 0.0}

    # -- producer side ---------------------------------------------------------
    def submit(self, req: Request):
        with self.cv:
            self.pending.append(req)
            self._admit_locked()
            self.cv.notify_all()

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()

    def _admit_locked(self):
        while self.pending:
            r = self.pending[0]
            b = request_bytes(self.n[r.mat], r.nrhs)
            if self.inflight_bytes + b > self.budget and self.inflight_bytes > 0:
                break
            self.pending.popleft()
            self.inflight_bytes += b
            self.peak_bytes = max(self.peak_bytes, self.inflight_bytes)
            self.admitted.append(r)

    # -- rounds ----------------------------------------------------------------
    def _take_round_locked(self):
        groups = {}        # (mat, tol) -> [requests]
        cols = {}
        used = set()
        keep = deque()
        # with a catalogue, a round's matrices (and those of the rounds
        # running) must fit its budget together; a round takes at least one
        room = None
        if self.cat is not None:
            room = self.cat.budget - sum(self.cat.expected_bytes(m) for m in self.busy)
            # requests on resident matrices first, and those that have waited
            # longer than max_wait_s; the others wait for their matrix's
            # requests to gather, so that one load serves many of them
            now = time.perf_counter()
            first = [r for r in self.admitted
                     if self.cat.is_resident(r.mat) or now - r.t_arrival > self.max_wait_s]
            ids = {id(r) for r in first}
            self.admitted = deque(first + [r for r in self.admitted if id(r) not in ids])
        round_bytes = 0
        while self.admitted:
            r = self.admitted.popleft()
            key = (r.mat, r.tol)
            if r.mat in self.busy or (r.mat in used and key not in groups):
                keep.append(r)
                continue
            if key not in groups:
                if len(used) >= self.max_mats:
                    keep.append(r)
                    continue
                if room is not None and r.mat not in used:
                    b = self.cat.expected_bytes(r.mat)
                    if used and round_bytes + b > room:
                        keep.append(r)
                        continue
                    round_bytes += b
                groups[key] = []
                cols[key] = 0
                used.add(r.mat)
            if cols[key] + r.nrhs > self.max_cols and groups[key]:
                keep.append(r)
                continue
            groups[key].append(r)
            cols[key] += r.nrhs
        # requests of one matrix in two tolerance classes: the matrix serves one
        # class this round
        by_mat = {}
        for (m, t) in list(groups):
            if m in by_mat:
                keep.extendleft(reversed(groups.pop((m, t))))
            else:
                by_mat[m] = t
        self.admitted = keep + self.admitted
        for m in by_mat:
            self.busy.add(m)
        return groups

    def _worker(self):
        torch = self.torch
        stream = torch.cuda.Stream()
        while True:
            with self.cv:
                while True:
                    groups = self._take_round_locked() if self.admitted else {}
                    if groups:
                        break
                    if self.closed and not self.admitted and not self.pending:
                        return
                    self.cv.wait(timeout=0.01)
            try:
                self._run_round(groups, stream)
            except Exception as ex:            # recorded; the loop keeps serving
                self.errors.append(repr(ex))
                for reqs in groups.values():
                    for r in reqs:
                        r.status = -1
                        r.t_done = time.perf_counter()
            with self.cv:
                for (m, _t), reqs in groups.items():
                    self.busy.discard(m)
                    for r in reqs:
                        self.inflight_bytes -= request_bytes(self.n[r.mat], r.nrhs)
                        self.done.append(r)
                self.rounds += 1
                self.round_sizes.append(sum(len(v) for v in groups.values()))
                self._admit_locked()
                self.cv.notify_all()

    def _run_round(self, groups, stream):
        """One round: per tolerance class, pack each matrix's requests into one
        column-major device block, run one batched solve over all of them, and
        hand every request its columns.  Device-resident requests (torch
        tensors) are packed with device copies and get views of the block as
        results; host requests go through a pinned staging block."""
        torch = self.torch
        by_tol = {}
        for (m, t), reqs in groups.items():
            by_tol.setdefault(t, []).append((m, reqs))
        acquired = []
        try:
            self._run_classes(by_tol, stream, acquired)
        finally:
            for m in acquired:
                self.cat.release(m)

    def _run_classes(self, by_tol, stream, acquired):
        torch = self.torch
        with torch.cuda.stream(stream):
            for tol, items in by_tol.items():
                t0 = time.perf_counter()
                mats, blocks, splits = [], [], []
                for m, reqs in items:
                    n = self.n[m]
                    cols = sum(r.nrhs for r in reqs)
                    if all(isinstance(r.B, torch.Tensor) for r in reqs):
                        dev = hss.empty_colmajor(n, cols, torch.float64)
                        c = 0
                        for r in reqs:
                            dev[:, c:c + r.nrhs].copy_(r.B, non_blocking=True)
                            c += r.nrhs
                    else:
                        host = torch.empty((cols, n), dtype=torch.float64, pin_memory=True)
                        c = 0
                        for r in reqs:
                            Bh = r.B.cpu().numpy() if isinstance(r.B, torch.Tensor) else r.B
                            host[c:c + r.nrhs].copy_(torch.from_numpy(np.ascontiguousarray(Bh.T)))
                            c += r.nrhs
                        dev = host.to("cuda", non_blocking=True).t()
                    mats.append(self.cat.acquire(m) if self.cat is not None else self.mats[m])
                    if self.cat is not None:
                        acquired.append(m)
                    blocks.append(dev)
                    splits.append(reqs)
                t1 = time.perf_counter()
                infos = hss.batch_solve(mats, blocks, prec=hss.F32, tol=tol,
                                        max_refine=self.max_refine, stream=stream)
                t2 = time.perf_counter()
                # host requests: one copy per block into pinned memory (the
                # caching host allocator reuses it), all issued before one wait
                staged = []
                for dev, reqs in zip(blocks, splits):
                    if all(isinstance(r.B, torch.Tensor) for r in reqs):
                        staged.append(None)
                        continue
                    ht = torch.empty(tuple(dev.t().shape), dtype=torch.float64, pin_memory=True)
                    ht.copy_(dev.t(), non_blocking=True)
                    staged.append(ht)
                if any(ht is not None for ht in staged):
                    stream.synchronize()
                for dev, reqs, info, ht in zip(blocks, splits, infos, staged):
                    host_out = ht.numpy().T if ht is not None else None
                    now = time.perf_counter()
                    c = 0
                    for r in reqs:
                        if isinstance(r.B, torch.Tensor):
                            r.X = dev[:, c:c + r.nrhs]
                        else:
                            r.X = host_out[:, c:c + r.nrhs]
                        r.eta = info["eta"][c:c + r.nrhs]
                        r.iters = info["iters"]
                        r.status = info["status"]
                        r.t_done = now
                        c += r.nrhs
                t3 = time.perf_counter()
                with self.cv:
                    self.phase_s["stage_in"] += t1 - t0
                    self.phase_s["solve"] += t2 - t1
                    self.phase_s["stage_out"] += t3 - t2

    def reserve_work(self):
        """Grow every resident matrix's work buffers to the widest group a
        round can give it (max_cols_per_group columns, refined FP32 solve)
        before requests arrive, so that rounds never allocate or retire them
        (a catalogue does it when it loads a matrix)."""
        from . import hss
        torch = self.torch
        if self.cat is not None:
            return
        for m in self.mats:
            B = hss.empty_colmajor(m.n, self.max_cols, torch.float64)
            B.fill_(1.0)
            m.solve(B, prec=hss.F32, tol=1e-10, max_refine=1, check=False)
            del B
        torch.cuda.synchronize()

    def start(self):
        self.reserve_work()
        self.threads = [threading.Thread(target=self._worker, daemon=True)
                        for _ in range(self.nworkers)]
        for t in self.threads:
            t.start()

    def join(self):
        for t in self.threads:
            t.join()


def run_stream(mats, requests, budget_bytes: int, workers: int = 2, pools=None):
    """Release ``requests`` at their arrival times (relative to now) into a
    server and wait for all of them.  Returns (server, wall seconds)."""
    ns = list(mats.n) if isinstance(mats, Catalogue) else [m.n for m in mats]
    for r in requests:
        if r.B is None:
            r.B = rhs_from_pool(r, pools) if pools is not None else rhs_for(r, ns[r.mat])
    srv = Server(mats, budget_bytes, workers=workers)
    srv.start()
    start = time.perf_counter()
    for r in requests:
        delay = start + r.t_arrival - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        r.t_arrival = time.perf_counter()
        srv.submit(r)
    srv.close()
    srv.join()
    return srv, time.perf_counter() - start


def latency_stats(reqs):
    """Latency percentiles over every completed request, whatever its status
    (a request that did not meet its tolerance still waited), with the count
    of those whose status is not HSS_OK beside them."""
    done = [r for r in reqs if r.t_done > 0.0]
    lat = np.array([r.t_done - r.t_arrival for r in done])
    if lat.size == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3),
            "completed": int(lat.size), "not_ok": int(sum(1 for r in done if r.status != 0))}
