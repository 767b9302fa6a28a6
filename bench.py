#!/usr/bin/env python3
"""Benchmark of the HSS solve and product path on one MI355X.

Workload: synthetic HSS matrix with n = 2^18, leaf size 128 (depth 11), HSS
rank k = 32 (orthonormal bases, core singular values 0.5 * 10^(-j/4),
D_i = 128 I + G / sqrt(128)), seeded; one right-hand side by default.

A step is one fresh-system solve to a normwise backward error <= 1e-10:
FP32 ULV factorization, FP32 solve, FP64 residual through the FP64 HSS
product, FP32 correction, until eta <= 1e-10 (eta is stated for every result).
Instances rotate (default 3) so the 256 MB last-level cache does not hold the
working set between steps.  ``value`` is fresh-system solves per second.

Also reported: the same step in plain FP64 (factor + solve + eta), resident
factor solves/s for both precisions, the FP64 product in GB/s of algorithmic
bytes at 1 and 32 right-hand sides, per-kernel times, the roofline of the
dominant kernel, and the FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

N, LEAF, RANK = 2 ** 18, 128, 32
HBM_PEAK_GBS = 8000.0
FP32_VEC_TFLOPS = 157.3
FP64_VEC_TFLOPS = 78.6
# HBM bytes per launch of the dominant kernels as they are now, from two
# rocprofv3 runs (FETCH_SIZE, then WRITE_SIZE) at the headline size, each
# scaled by what the counter reads for a plain device copy of known size
# (x2.0 and x1.0); reported as the roofline line's "traffic".
MEASURED_TRAFFIC = {"ulv_factor_leaf_f32": 543_217_426, "ulv_factor_leaf_f64": 1_562_816_968}
METRIC = "HSS solves/s & matmul GB/s, n=2^18 k=32; FP32+IR vs FP64 at 1e-10 bkwd err"


def gen_entries(n_leaf, m, k):
    """Generator entries of the uniform tree: leaves m^2 + 2mk, non-root
    internal 2 * (2k x k), internal 2 * (k x k)."""
    return n_leaf * (m * m + 2 * m * k) + (n_leaf - 2) * 2 * (2 * k * k) + (n_leaf - 1) * 2 * k * k


def householder_flops(m, ku, kv):
    """Flops of Step 1 on one block as the kernels implement it (unblocked
    Householder QL of U' applied to D' and U', LQ of the leading e rows applied
    to the trailing rows and to V'): 4 flops per (reflector entry x column)."""
    e = max(m - ku, 0)
    f = 0
    if e > 0:
        for j in range(ku):
            L = e + j + 1
            f += 4 * L * (m + j)
    for i in range(e):
        L = m - i
        f += 4 * L * (m - i - 1 + kv)
    return f


def kernel_units(name, n, m, k, r):
    """(bound, algorithmic units per launch, unit) for the kernels at the
    uniform tree with nleaf leaves; bytes for HBM-bound kernels, flops else."""
    nleaf = n // m
    ew = 4 if name.endswith("f32") else 8
    if name.startswith("ulv_factor_leaf"):
        return ("alu", householder_flops(m, k, k) * nleaf, "flop")
    if name.startswith("mm_leaf_out"):
        return ("hbm", (nleaf * (m * m + m * k) + 2 * n * r + nleaf * k * r) * ew, "byte")
    if name.startswith("mm_leaf_up"):
        return ("hbm", (nleaf * m * k + n * r + nleaf * k * r) * ew, "byte")
    if name.startswith("sv_fwd_leaf") or name.startswith("sv_bwd_leaf"):
        return ("hbm", (nleaf * (m * m + 2 * m * k) + 2 * n * r) * ew, "byte")
    return (None, None, None)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--max-refine", type=int, default=2,
                    help="refinement steps enqueued per solve, each gated on the device by "
                         "the backward error before it (one is needed on this family)")
    ap.add_argument("--instances", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "batch", "serve", "construct", "cpu"],
                    help="headline: one n=2^18 system (default); batch: 512 uneven instances "
                         "in level-batched launches; serve: Poisson request stream; "
                         "construct: dense-to-HSS construction of the n=16384 Cauchy-like "
                         "matrix; cpu: the FP64 oracle timed on the host for every workload "
                         "(no GPU)")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-resident", type=float, default=1.0,
                    help="serving: device budget for resident matrices as a fraction of the "
                         "whole catalogue (below 1: created and evicted on demand, LRU)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one plain device copy of this many bytes (a reference "
                         "kernel of known traffic for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this "
              "build (independent instances shard across GPUs without communication: run one "
              "process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "cpu":
        return bench_cpu(args)

    import numpy as np
    import torch

    from paper_1909_07909_amd import hss, inputs

    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "construct":
        return bench_construct(args)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    r = args.nrhs
    lo = hss.plan_leaf_offsets(N, LEAF)
    p = hss.plan_depth(N, LEAF)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"[bench] n={N} leaf={LEAF} p={p} k={RANK} r={r} instances={args.instances}")
    mats, B0 = [], []
    for i in range(args.instances):
        g = inputs.synthetic_hss(lo, RANK, seed=2 + 1000 * i)
        mats.append(hss.HSSMatrix(g))
        b = inputs.rhs(N, r, 3 + i)
        B0.append(torch.from_numpy(np.ascontiguousarray(b.T)).to(dev).t())
        del g
    G = mats[0].query(hss.Q_GEN_ENTRIES)
    assert G == gen_entries(2 ** p, LEAF, RANK)
    log(f"[bench] created {args.instances} instances, {G} generator entries each")
    work = [hss.empty_colmajor(N, r, torch.float64) for _ in mats]
    # ||A||_2 is estimated once per matrix by hss_create (16 power steps, 32
    # products); it is part of creating the matrix, not of a step
    mr = args.max_refine

    def step_fresh(i, prec, tol, rep, max_refine=None):
        """A fresh system: factor and refined solve in one call
        (hss_ulv_factor_solve; in FP64 the first forward sweep overlapped
        with the factorization)."""
        A = mats[i % len(mats)]
        W = work[i % len(mats)]
        W.copy_(B0[i % len(mats)])
        if prec == hss.F32:
            return A.factor_solve(W, prec=hss.F32, tol=tol, max_refine=mr if max_refine is None
                                  else max_refine, sync=False, report=rep)
        return A.factor_solve(W, prec=hss.F64, want_eta=True, sync=False, report=rep)

    def step_fresh_separate(i, prec, tol, rep):
        """The same as two calls: hss_ulv_factor, then hss_ulv_solve."""
        A = mats[i % len(mats)]
        W = work[i % len(mats)]
        W.copy_(B0[i % len(mats)])
        A.factor(prec)
        if prec == hss.F32:
            return A.solve(W, prec=hss.F32, tol=tol, max_refine=mr, sync=False, report=rep)
        return A.solve(W, prec=hss.F64, want_eta=True, sync=False, report=rep)

    def step_resident(i, prec, tol, rep):
        A = mats[i % len(mats)]
        W = work[i % len(mats)]
        W.copy_(B0[i % len(mats)])
        if prec == hss.F32:
            return A.solve(W, prec=hss.F32, tol=tol, max_refine=mr, sync=False, report=rep)
        return A.solve(W, prec=hss.F64, want_eta=True, sync=False, report=rep)

    def timed(fn, steps, warmup, *a, ncols=r):
        """Steps are enqueued back to back (the solves are stream-ordered and
        write their reports on the device); one synchronisation at the end."""
        reps = [hss.SolveReport(ncols) for _ in range(max(steps, warmup))]
        for i in range(warmup):
            fn(i, *a, reps[i])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            fn(i, *a, reps[i])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        etas = []
        for i in range(steps):
            info = reps[i].result()
            if info["status"] != hss.HSS_OK:
                raise hss.HSSError(info["status"], "bench step")
            etas.append((info["eta_max"], info["iters"]))
        return dt, etas

    K, W = args.steps, args.warmup
    # headline: FP32 + refinement, fresh systems
    t32, e32 = timed(step_fresh, K, W, hss.F32, 1e-10)
    log(f"[bench] fresh FP32+IR: {t32*1e3:.3f} ms/solve, eta_max {max(e for e, _ in e32):.2e}, "
        f"iters {max(i for _, i in e32)}")
    # the same with ten refinement steps enqueued (the library's default): the
    # steps after convergence are gated off on the device but still launched
    t32_10, e32_10 = timed(lambda i, p, t, rp: step_fresh(i, p, t, rp, 10), K, W, hss.F32, 1e-10)
    log(f"[bench] fresh FP32+IR, max_refine 10: {t32_10*1e3:.3f} ms/solve")
    t64, e64 = timed(step_fresh, K, W, hss.F64, 0.0)
    log(f"[bench] fresh FP64   : {t64*1e3:.3f} ms/solve, eta_max {max(e for e, _ in e64):.2e}")
    ts32, _ = timed(step_fresh_separate, K, W, hss.F32, 1e-10)
    ts64, _ = timed(step_fresh_separate, K, W, hss.F64, 0.0)
    log(f"[bench] fresh as separate factor + solve calls: FP32+IR {ts32*1e3:.3f} ms, "
        f"FP64 {ts64*1e3:.3f} ms")

    def graph_rate(prec, tol):
        """The fresh step (copy of the right-hand side, factorization, solve
        with its device-gated refinement, device-written report) captured once
        per instance in a HIP graph and replayed round robin."""
        reps_g = [hss.SolveReport(r) for _ in mats]
        fns = [lambda i=i: step_fresh(i, prec, tol, reps_g[i]) for i in range(len(mats))]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for f in fns:
                f()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graphs = []
        for f in fns:
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr):
                f()
            graphs.append(gr)
        torch.cuda.synchronize()
        for i in range(W):
            graphs[i % len(graphs)].replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(K):
            graphs[i % len(graphs)].replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / K
        infos = [rp.result() for rp in reps_g]
        del graphs
        for info in infos:
            if info["status"] != hss.HSS_OK:
                raise hss.HSSError(info["status"], "bench graph step")
        return dt, max(info["eta_max"] for info in infos), max(info["iters"] for info in infos)

    g32, ge32, gi32 = graph_rate(hss.F32, 1e-10)
    g64, ge64, _ = graph_rate(hss.F64, 0.0)
    log(f"[bench] graph replay: fresh FP32+IR {g32*1e3:.3f} ms/solve (eta_max {ge32:.2e}, "
        f"iters {gi32}), FP64 {g64*1e3:.3f} ms/solve")
    # resident factors (both precisions factored)
    for A in mats:
        A.factor(hss.F32)
        A.factor(hss.F64)
    torch.cuda.synchronize()
    rt32, re32 = timed(step_resident, K, W, hss.F32, 1e-10)
    rt64, re64 = timed(step_resident, K, W, hss.F64, 0.0)
    log(f"[bench] resident FP32+IR {rt32*1e3:.3f} ms, FP64 {rt64*1e3:.3f} ms")

    # the same fresh-system solves with a block of 32 right-hand sides
    wide = None
    if r == 1:
        rw = 32
        Bw = [torch.from_numpy(np.ascontiguousarray(inputs.rhs(N, rw, 50 + i).T)).to(dev).t()
              for i in range(len(mats))]
        Ww = [hss.empty_colmajor(N, rw, torch.float64) for _ in mats]

        def step_wide(i, prec, tol, rep):
            A = mats[i % len(mats)]
            X = Ww[i % len(mats)]
            X.copy_(Bw[i % len(mats)])
            A.factor(prec)
            if prec == hss.F32:
                return A.solve(X, prec=hss.F32, tol=tol, max_refine=mr, sync=False, report=rep)
            return A.solve(X, prec=hss.F64, want_eta=True, sync=False, report=rep)

        # launch choices for 32-column products and sweeps, timed on this
        # shape (hss_autotune) and used by every later call on it
        tuned = {"fp32": mats[0].autotune(rw, hss.F32), "fp64": mats[0].autotune(rw, hss.F64)}
        log("[bench] autotuned r=32: " + ", ".join(
            f"{k}: product {'wide' if v['product_wide'] else 'mailbox'} "
            f"({v['product_us'][0]:.0f} / {v['product_us'][1]:.0f} us), sweep cpw {v['solve_cpw']} "
            f"({v['solve_us'][0]:.0f} / {v['solve_us'][1]:.0f} us)" for k, v in tuned.items()))
        kw = max(K // 2, 3)
        w32, ew32 = timed(step_wide, kw, W, hss.F32, 1e-10, ncols=rw)
        w64, ew64 = timed(step_wide, kw, W, hss.F64, 0.0, ncols=rw)
        wide = {"nrhs": rw, "steps": kw,
                "fp32ir": {"solves_per_s": round(1.0 / w32, 2), "ms": round(w32 * 1e3, 3),
                           "eta_max": max(e for e, _ in ew32),
                           "refine_iters_max": max(i for _, i in ew32)},
                "fp64": {"solves_per_s": round(1.0 / w64, 2), "ms": round(w64 * 1e3, 3),
                         "eta_max": max(e for e, _ in ew64)},
                "ratio_fp32ir_over_fp64": round(w64 / w32, 3),
                "autotuned": tuned}
        log(f"[bench] fresh r={rw}: FP32+IR {w32*1e3:.3f} ms (eta_max "
            f"{wide['fp32ir']['eta_max']:.2e}), FP64 {w64*1e3:.3f} ms (eta_max "
            f"{wide['fp64']['eta_max']:.2e})")
        del Bw, Ww

    # FP64 product at 1 and 32 right-hand sides (GB/s of algorithmic bytes)
    mm = {}
    for rr in (1, 32):
        Xs = [hss.empty_colmajor(N, rr, torch.float64) for _ in mats]
        Ys = [hss.empty_colmajor(N, rr, torch.float64) for _ in mats]
        for x in Xs:
            x.normal_()
        for i in range(W):
            mats[i % len(mats)].matmul(Xs[i % len(mats)], Ys[i % len(mats)])
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for i in range(K):
            mats[i % len(mats)].matmul(Xs[i % len(mats)], Ys[i % len(mats)])
        ev1.record(stream)
        torch.cuda.synchronize()
        us = ev0.elapsed_time(ev1) * 1e3 / K
        byt = (G + 2 * N * rr) * 8
        # the same products captured once per instance in a HIP graph and replayed
        graphs = []
        for i in range(len(mats)):
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr):
                mats[i].matmul(Xs[i], Ys[i])
            graphs.append(gr)
        for i in range(W):
            graphs[i % len(mats)].replay()
        torch.cuda.synchronize()
        ev0.record(stream)
        for i in range(K):
            graphs[i % len(mats)].replay()
        ev1.record(stream)
        torch.cuda.synchronize()
        gus = ev0.elapsed_time(ev1) * 1e3 / K
        del graphs
        mm[f"r{rr}"] = {"us": round(us, 2), "algorithmic_bytes": byt,
                        "gbps": round(byt / us / 1e3, 1),
                        "frac_hbm_peak": round(byt / us / 1e3 / HBM_PEAK_GBS, 4),
                        "graph_replay": {"us": round(gus, 2), "gbps": round(byt / gus / 1e3, 1),
                                         "frac_hbm_peak": round(byt / gus / 1e3 / HBM_PEAK_GBS, 4)}}
        log(f"[bench] FP64 matmul r={rr}: {us:.1f} us, {byt / us / 1e3:.1f} GB/s; "
            f"graph replay {gus:.1f} us, {byt / gus / 1e3:.1f} GB/s")

    # what the ||A||_2 estimate of hss_create costs (16 power steps: 16
    # products with A and 16 with A^T at one column)
    xv = hss.empty_colmajor(N, 1, torch.float64).normal_()
    yv = hss.empty_colmajor(N, 1, torch.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(16):
        mats[0].matmul(xv, yv)
        mats[0].matmul(yv, xv, op=hss.OP_T)
    torch.cuda.synchronize()
    norm_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] ||A||_2 estimate (16 power steps at create): {norm_ms:.2f} ms")

    # per-kernel times (events around every launch) of the headline step, the
    # FP64 step and the FP64 product
    def kernel_times(fn, reps):
        hss.timing_enable(True)
        hss.timing_report(reset=True)
        for i in range(reps):
            fn(i)
        torch.cuda.synchronize()
        rep = hss.timing_report(reset=True)
        hss.timing_enable(False)
        rep.sort(key=lambda d: -d["total_ms"])
        return rep

    krep = hss.SolveReport(r)
    rep = kernel_times(lambda i: step_fresh(i, hss.F32, 1e-10, krep), K)
    kernels = [{"kernel": d["kernel"], "launches_per_step": d["launches"] / K,
                "ms_per_step": round(d["total_ms"] / K, 4)} for d in rep]
    log("[bench] kernels per FP32+IR step: " + ", ".join(
        f"{d['kernel']} {d['ms_per_step']:.3f}ms" for d in kernels[:10]))
    rep64 = kernel_times(lambda i: step_fresh(i, hss.F64, 0.0, krep), K)
    log("[bench] kernels per FP64 step: " + ", ".join(
        f"{d['kernel']} {d['total_ms'] / K:.3f}ms" for d in rep64[:10]))
    for rr in (1, 32):
        Xm = hss.empty_colmajor(N, rr, torch.float64).normal_()
        Ym = hss.empty_colmajor(N, rr, torch.float64)
        repm = kernel_times(lambda i: mats[i % len(mats)].matmul(Xm, Ym), K)
        mm[f"r{rr}"]["kernels_us"] = {d["kernel"]: round(d["total_ms"] / K * 1e3, 2)
                                      for d in repm}
        log(f"[bench] matmul r={rr} kernels (us): " + ", ".join(
            f"{d['kernel']} {d['total_ms'] / K * 1e3:.1f}" for d in repm))
    roof = None
    for d in rep:
        bound, units, unit = kernel_units(d["kernel"], N, LEAF, RANK, r)
        if bound is None:
            continue
        avg_s = d["total_ms"] / d["launches"] / 1e3
        if bound == "hbm":
            ach = units / avg_s / 1e9
            roof = {"kernel": d["kernel"], "bound": "hbm", "achieved": round(ach, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": None, "avg_launch_us": round(avg_s * 1e6, 2)}
        else:
            pk = FP32_VEC_TFLOPS if d["kernel"].endswith("f32") else FP64_VEC_TFLOPS
            ach = units / avg_s / 1e12
            roof = {"kernel": d["kernel"], "bound": "alu", "achieved": round(ach, 3),
                    "peak": pk, "unit": "TFLOP/s", "frac": round(ach / pk, 4),
                    "traffic": MEASURED_TRAFFIC.get(d["kernel"]),
                    "avg_launch_us": round(avg_s * 1e6, 2)}
        break

    had = hadamard_measure(log)
    cons = construct_measure(log)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(lo, r)
        log(f"[bench] cpu oracle: {cpu}")

    out = {
        "metric": METRIC, "value": round(1.0 / t32, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": round(t32 * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64ir", "data": "synthetic",
        "config": {"workload": f"HSS fresh-system solve to eta<=1e-10, n={N}, leaf={LEAF}, "
                               f"depth={p}, k={RANK}, nrhs={r}, synthetic generators, "
                               f"{args.instances} rotating instances, max_refine={mr} "
                               f"(device-gated steps, no host synchronisation in a step)",
                   "n": N, "leaf": LEAF, "k": RANK, "nrhs": r, "max_refine": mr},
        "eta_max": max(e for e, _ in e32), "refine_iters_max": max(i for _, i in e32),
        "fp32ir_max_refine10": {"solves_per_s": round(1.0 / t32_10, 2),
                                "ms": round(t32_10 * 1e3, 4),
                                "eta_max": max(e for e, _ in e32_10)},
        "norm2_note": "||A||_2 for eta is estimated once per matrix by hss_create (16 power "
                      "steps = 32 FP64 products) and is not part of a step",
        "norm2_estimate_ms": round(norm_ms, 3),
        "fp64_solves_per_s": round(1.0 / t64, 2), "fp64_eta_max": max(e for e, _ in e64),
        "ratio_fp32ir_over_fp64": round(t64 / t32, 3),
        "resident_solves_per_s": {"fp32ir": round(1.0 / rt32, 2), "fp64": round(1.0 / rt64, 2)},
        "separate_calls": {"fp32ir_solves_per_s": round(1.0 / ts32, 2), "fp32ir_ms": round(ts32 * 1e3, 4),
                           "fp64_solves_per_s": round(1.0 / ts64, 2), "fp64_ms": round(ts64 * 1e3, 4)},
        "graph_replay": {"fp32ir_solves_per_s": round(1.0 / g32, 2), "fp32ir_ms": round(g32 * 1e3, 4),
                         "fp32ir_eta_max": ge32, "fp32ir_iters": gi32,
                         "fp64_solves_per_s": round(1.0 / g64, 2), "fp64_ms": round(g64 * 1e3, 4),
                         "fp64_eta_max": ge64},
        "fresh_nrhs32": wide,
        "matmul_fp64": mm,
        "hadamard": had,
        "compress": had.pop("compress", None),
        "construct": cons,
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels[:12],
    }
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


def construct_measure(log, reps=3, n=16384, leaf=128, eps=1e-10):
    """Dense-to-HSS construction (hss_construct_dense) of the Cauchy-like
    kernel matrix of the ragged-rank workload, n = 16384, leaf 128,
    eps = 1e-10 (relative to each block's sigma_1), the dense matrix resident
    in HBM: whole call time, per-kernel times, and the leaf-level truncation
    (the O(n^2) part) against its Householder-QR flops."""
    import numpy as np
    import torch

    from paper_1909_07909_amd import hss
    rng = np.random.default_rng(1)
    x = torch.from_numpy(np.sort(rng.uniform(0.0, 1.0, n))).cuda()
    d = (x[:, None] - x[None, :]) / 0.05
    A = 1.0 / (1.0 + d * d)
    A.diagonal().add_(1e-2)
    Ad = A.t()          # symmetric: the column-major view of the same matrix
    del d
    lo = hss.plan_leaf_offsets(n, leaf)
    H = hss.HSSMatrix.from_dense(Ad, leaf_off=lo, eps=eps)   # warm-up
    ku = H.ku.copy()
    del H
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        H = hss.HSSMatrix.from_dense(Ad, leaf_off=lo, eps=eps)
        del H
    torch.cuda.synchronize()
    call_ms = (time.perf_counter() - t0) * 1e3 / reps
    hss.timing_enable(True)
    hss.timing_report(reset=True)
    H = hss.HSSMatrix.from_dense(Ad, leaf_off=lo, eps=eps)
    torch.cuda.synchronize()
    rep = hss.timing_report(reset=True)
    hss.timing_enable(False)
    del H, A, Ad
    m = np.diff(lo)
    # Householder QR of H^T (N x r, N = n - r columns of the block row):
    # 2 N r^2 - 2 r^3 / 3 flops, a row side and a column side per leaf
    flops = float(np.sum(2 * (2.0 * (n - m) * m * m - 2.0 * m ** 3 / 3.0)))
    kt = {d["kernel"]: d for d in rep}
    leaf_ms = kt["construct_trunc_leaf"]["total_ms"]
    tf = flops / (leaf_ms * 1e-3) / 1e12
    out = {"workload": f"Cauchy-like kernel, n={n}, leaf={leaf}, eps={eps:g}",
           "call_ms": round(call_ms, 3),
           "mean_rank": round(float(np.mean(ku[1:])), 2), "max_rank": int(ku.max()),
           "kernels_ms": {d["kernel"]: round(d["total_ms"], 3) for d in rep
                          if d["kernel"].startswith("construct")},
           "trunc_leaf": {"ms": round(leaf_ms, 3), "algorithmic_flops": flops,
                          "tflops": round(tf, 2), "frac_fp64_vector_peak": round(tf / 78.6, 4)}}
    log(f"[bench] construct n={n}: {call_ms:.2f} ms per call (mean rank "
        f"{out['mean_rank']}); leaf truncation {leaf_ms:.2f} ms, {tf:.2f} TFLOP/s")
    return out


def bench_construct(args):
    """The construction workload alone: one JSON line."""
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    c = construct_measure(log, reps=max(args.steps, 1))
    out = {"metric": "dense-to-HSS constructions/s [construction workload]",
           "value": round(1e3 / c["call_ms"], 3), "unit": "constructions/s", "n_gpus": 1,
           "steps": max(args.steps, 1), "warmup": 1, "ms_per_step": c["call_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {"workload": c["workload"]}, "construct": c}
    line = json.dumps(out)
    print(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


def hadamard_measure(log, reps=5, ka=8, kb=4):
    """The Hadamard product of two n=2^18, leaf-128 matrices of ranks ka and kb
    (the result has rank ka*kb = 32, the headline shape): per-kernel times
    from events around each launch, against the generator bytes each kernel
    reads and writes, and the whole hss_hadamard call (which also makes the
    FP32 copy and the ||C||_2 estimate and synchronizes)."""
    import numpy as np
    import torch

    from paper_1909_07909_amd import hss, inputs
    lo = hss.plan_leaf_offsets(N, LEAF)
    A = hss.HSSMatrix(inputs.synthetic_hss(lo, ka, seed=40))
    B = hss.HSSMatrix(inputs.synthetic_hss(lo, kb, seed=41))
    C = A.hadamard(B)   # warm-up
    sa, sb, sc = A.packed_sizes(), B.packed_sizes(), C.packed_sizes()
    del C
    torch.cuda.synchronize()
    hss.timing_enable(True)
    hss.timing_report(reset=True)
    t0 = time.perf_counter()
    for _ in range(reps):
        C = A.hadamard(B)
        del C
    call_ms = (time.perf_counter() - t0) * 1e3 / reps
    rep = {d["kernel"]: d for d in hss.timing_report(reset=True)}
    hss.timing_enable(False)
    diag_bytes = 8 * (sa["D"] + sb["D"] + sc["D"])
    rest = ("U", "V", "R", "W", "B12", "B21")
    gen_bytes = 8 * sum(sa[k] + sb[k] + sc[k] for k in rest)
    out = {"workload": f"C = A o B, n={N}, leaf={LEAF}, ranks {ka} x {kb} -> {ka * kb}",
           "call_ms": round(call_ms, 3)}
    for name, byt in (("hadamard_diag", diag_bytes), ("hadamard_gen", gen_bytes)):
        d = rep.get(name)
        if d is None:
            continue
        us = d["total_ms"] / d["launches"] * 1e3
        out[name] = {"us": round(us, 2), "algorithmic_bytes": byt,
                     "gbps": round(byt / us / 1e3, 1),
                     "frac_hbm_peak": round(byt / us / 1e3 / HBM_PEAK_GBS, 4)}
    tot_us = sum(out[k]["us"] for k in ("hadamard_diag", "hadamard_gen") if k in out)
    out["kernels_us"] = round(tot_us, 2)
    out["gbps"] = round((diag_bytes + gen_bytes) / tot_us / 1e3, 1)
    log(f"[bench] hadamard: kernels {tot_us:.1f} us ({out['gbps']} GB/s), "
        f"whole call {call_ms:.2f} ms")

    # recompression of the product (its ranks are ka*kb, more than the
    # singular values of its blocks need) at tau = 1e-8 ||C||_2
    C = A.hadamard(B)
    tau = 1e-8 * C.norm2()
    Cc = C.compress(tau=tau)   # warm-up
    del Cc
    torch.cuda.synchronize()
    hss.timing_enable(True)
    hss.timing_report(reset=True)
    t0 = time.perf_counter()
    for _ in range(reps):
        Cc = C.compress(tau=tau)
    call_c = (time.perf_counter() - t0) * 1e3 / reps
    repc = hss.timing_report(reset=True)
    hss.timing_enable(False)
    k_in = float(np.mean(C.ku[1:]))
    k_out = float(np.mean(Cc.ku[1:]))
    comp = {"workload": f"compress C (n={N}, leaf={LEAF}, rank {ka * kb}) at tau = 1e-8 ||C||_2",
            "call_ms": round(call_c, 3), "mean_rank_in": round(k_in, 2),
            "mean_rank_out": round(k_out, 2),
            "max_rank_out": int(max(Cc.ku.max(), Cc.kv.max())),
            "kernels_ms": {d["kernel"]: round(d["total_ms"] / reps, 3)
                           for d in repc if d["kernel"].startswith("compress")}}
    log(f"[bench] compress: {call_c:.2f} ms per call, mean rank {k_in:.1f} -> {k_out:.1f}; "
        + ", ".join(f"{k} {v:.2f} ms" for k, v in comp["kernels_ms"].items()))
    out["compress"] = comp
    return out


def _emit(out, args):
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


def _gen_batch_instance(child):
    import numpy as np

    from paper_1909_07909_amd import hss, inputs
    r = np.random.default_rng(child)
    n = 64 * int(r.integers(32, 513))
    k = int(r.choice([8, 16, 24]))
    return inputs.synthetic_hss(hss.plan_leaf_offsets(n, 64), k, seed=child)


def bench_batch(args):
    """512 independent instances, n = 64 * U{32..512}, leaf 64, k in {8,16,24},
    8 right-hand sides each; all factored and solved with one launch per tree
    level across the instances, FP32+IR (eta <= 1e-10) and FP64."""
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np
    import torch

    from paper_1909_07909_amd import hss, inputs
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    count, r = 512, 8
    kids = np.random.SeedSequence(3).spawn(count)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=16) as ex:
        gens = list(ex.map(_gen_batch_instance, kids, chunksize=8))
    log(f"[bench-batch] generated {count} instances in {time.perf_counter() - t0:.1f} s, "
        f"sum n = {sum(g.n for g in gens)}")
    mats = [hss.HSSMatrix(g) for g in gens]
    G = sum(m.query(hss.Q_GEN_ENTRIES) for m in mats)
    B0 = [torch.from_numpy(np.ascontiguousarray(inputs.rhs(g.n, r, 7 + j).T)).cuda().t()
          for j, g in enumerate(gens)]
    del gens
    work = [b.clone().t().contiguous().t() for b in B0]
    for m in mats:
        m.norm2()

    def step(prec):
        for w, b in zip(work, B0):
            w.copy_(b)
        hss.batch_factor(mats, prec)
        if prec == hss.F32:
            return hss.batch_solve(mats, work, prec=hss.F32, tol=1e-10, max_refine=args.max_refine)
        return hss.batch_solve(mats, work, prec=hss.F64, want_eta=True)

    res = {}
    for name, prec in (("fp32ir", hss.F32), ("fp64", hss.F64)):
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            infos = step(prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        res[name] = {"ms_per_step": round(dt * 1e3, 3), "systems_per_s": round(count / dt, 1),
                     "eta_max": max(i["eta_max"] for i in infos),
                     "iters_max": max(i["iters"] for i in infos)}
        log(f"[bench-batch] {name}: {dt * 1e3:.2f} ms per {count} systems, "
            f"eta_max {res[name]['eta_max']:.2e}")
    # per-kernel event timings of one step of each precision
    for name, prec in (("fp32ir", hss.F32), ("fp64", hss.F64)):
        hss.timing_enable(True)
        hss.timing_report(reset=True)
        step(prec)
        torch.cuda.synchronize()
        rep = sorted(hss.timing_report(reset=True), key=lambda d: -d["total_ms"])
        hss.timing_enable(False)
        res[name]["kernels_ms"] = {d["kernel"]: round(d["total_ms"], 3) for d in rep[:12]}
        log(f"[bench-batch] {name} kernels: " + ", ".join(
            f"{d['kernel']} {d['total_ms']:.2f}ms/{d['launches']}" for d in rep[:12]))
    # level-batched FP64 product, 8 columns each
    Ys = [hss.empty_colmajor(m.n, r, torch.float64) for m in mats]
    for _ in range(args.warmup):
        hss.batch_matmul(mats, B0, Ys)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        hss.batch_matmul(mats, B0, Ys)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    nsum = sum(m.n for m in mats)
    byt = (G + 2 * nsum * r) * 8
    res["matmul_fp64"] = {"ms": round(dt * 1e3, 3), "gbps": round(byt / dt / 1e9, 1)}
    out = {"metric": METRIC + " [batching workload]", "value": res["fp32ir"]["systems_per_s"],
           "unit": "systems/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["fp32ir"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64ir", "data": "synthetic",
           "config": {"workload": f"{count} HSS instances, n=64*U{{32..512}} (sum {nsum}), leaf 64, "
                                  f"k in {{8,16,24}}, nrhs={r}, factor + solve to eta<=1e-10, "
                                  "one launch per tree level across instances"},
           "fp64": res["fp64"], "fp32ir": res["fp32ir"], "matmul_fp64": res["matmul_fp64"],
           "ratio_fp32ir_over_fp64": round(res["fp64"]["ms_per_step"] / res["fp32ir"]["ms_per_step"], 3),
           "roofline": None, "cpu_baseline": None}
    _emit(out, args)


def bench_serve(args):
    """Poisson stream of solve requests against a catalogue of resident,
    FP32-factored matrices (n log-uniform in [4096, 2^20], k in {16,32,64},
    leaf 128), tolerance 1e-6 or 1e-10 at equal odds, 1-16 columns."""
    import numpy as np
    import torch

    from paper_1909_07909_amd import hss, serve
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    specs = serve.draw_catalogue(16, seed=4)
    t0 = time.perf_counter()
    gens = serve.build_catalogue(specs, seed=4, workers=16)
    log(f"[bench-serve] catalogue {specs} generated in {time.perf_counter() - t0:.1f} s")
    mats = [hss.HSSMatrix(g) for g in gens]
    t0 = time.perf_counter()
    for m in mats:
        m.factor(hss.F32)
        m.norm2()
    torch.cuda.synchronize()
    log(f"[bench-serve] factored in {time.perf_counter() - t0:.2f} s")
    cat = None
    if args.serve_resident < 1.0:
        # bounded residency: a catalogue with room for that fraction of the
        # matrices' measured bytes, loading and evicting them on demand
        total = sum(m.query(hss.Q_RESIDENT_BYTES) for m in mats)
        for m in mats:
            m.close()
        mats = cat = serve.Catalogue(gens, budget_bytes=int(args.serve_resident * total))
        log(f"[bench-serve] catalogue budget {cat.budget / 2**30:.1f} GiB of {total / 2**30:.1f} GiB")
    del gens
    pools = serve.rhs_pools(mats, device=True)   # request blocks resident in HBM
    warm = serve.poisson_requests(args.serve_rate, 0.2, len(mats), seed=40)
    serve.run_stream(mats, warm, budget_bytes=24 << 30, workers=2, pools=pools)
    reqs = serve.poisson_requests(args.serve_rate, args.serve_seconds, len(mats), seed=41)
    srv, wall = serve.run_stream(mats, reqs, budget_bytes=24 << 30, workers=2, pools=pools)
    ok = [r for r in srv.done if r.status == 0]
    lat = serve.latency_stats(srv.done)
    good = all(r.eta.max() <= r.tol for r in ok)
    cols = sum(r.nrhs for r in ok)
    log(f"[bench-serve] {len(ok)}/{len(reqs)} requests in {wall:.2f} s, {lat}, all within tol: {good}")
    out = {"metric": METRIC + " [serving workload]", "value": round(len(ok) / wall, 1),
           "unit": "solves/s", "n_gpus": 1, "steps": len(reqs), "warmup": len(warm),
           "ms_per_step": round(wall / max(len(ok), 1) * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64ir", "data": "synthetic",
           "config": {"workload": f"Poisson {args.serve_rate:.0f} req/s for {args.serve_seconds} s, "
                                  f"16 matrices n log-uniform [4096, 2^20] ({'all resident' if cat is None else f'{args.serve_resident:.0%} resident, LRU'}), k in {{16,32,64}}, "
                                  "leaf 128, tol 1e-6 / 1e-10, 1-16 rhs, request blocks in HBM"},
           "latency": lat, "rhs_columns_per_s": round(cols / wall, 1),
           "all_within_tol": good, "rounds": srv.rounds,
           "mean_requests_per_round": round(float(np.mean(srv.round_sizes)), 2),
           "peak_inflight_bytes": srv.peak_bytes,
           "worker_phase_s": {k: round(v, 3) for k, v in srv.phase_s.items()},
           "resident_bytes": (cat.resident_bytes() if cat is not None else
                              int(sum(m.query(hss.Q_RESIDENT_BYTES) for m in mats))),
           "catalogue": cat.stats() if cat is not None else None,
           "errors": srv.errors[:3], "roofline": None, "cpu_baseline": None}
    _emit(out, args)


def _host_cores():
    """Host cores available to this process (the machine's CPU share)."""
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def _median_time(fn, reps, warm=1):
    """Median wall time of fn() over reps runs after warm untimed runs."""
    import numpy as np
    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), [round(t, 4) for t in ts]


def cpu_baseline(lo, r, reps=3):
    """The FP64 oracle (literal recursive ULV of Sec. 4.3, unoptimized
    reference) on the host: the headline step, one fresh-system solve
    (factorization and solve) of the n=2^18 instance, median of `reps` runs
    after one warm-up, BLAS threads = the host cores available.  The full
    table over every workload and at one thread is bench.py --workload cpu."""
    from threadpoolctl import threadpool_limits

    from oracle.hss import HSS
    from oracle.ulv import solve
    from paper_1909_07909_amd import inputs
    cores = _host_cores()
    g = inputs.synthetic_hss(lo, RANK, seed=2)
    H = HSS.from_packed(g)
    b = inputs.rhs(N, r, 3)
    with threadpool_limits(limits=cores):
        med, ts = _median_time(lambda: solve(H, b), reps)
    return {"value": round(1.0 / med, 4), "unit": "solves/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"fresh FP64 solve (literal recursive ULV, factor+solve) of the n={N}, "
                      f"k={RANK}, nrhs={r} instance, median of {reps} after 1 warm-up "
                      f"({ts} s); ||A||_2 for eta is not part of it (the oracle's power method, "
                      f"50 steps, takes about 100 products)"}


def bench_cpu(args):
    """The FP64 oracle timed on the host for every workload, all cores and
    one core, median of 5 runs after one warm-up: products at 1 and 32 (64)
    right-hand sides and fresh factor+solve for the small-parity, ragged-rank
    and headline workloads, and factor+solve of 32 instances of the batching
    workload.  The oracle is the unoptimized reference implementation (plain
    NumPy/SciPy recursion), not a tuned CPU library."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    from cauchy_fixture import cauchy_hss
    from oracle import tree
    from oracle.hss import HSS
    from oracle.matvec import matvec
    from oracle.ulv import solve
    from paper_1909_07909_amd import inputs
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    cores = _host_cores()
    reps = 5
    cases = []
    g0 = inputs.synthetic_hss(tree.leaf_offsets(1024, 64), 8, seed=0)
    cases.append(("c0 n=1024 m=64 k=8", HSS.from_packed(g0), [1, 16], 16))
    log("[cpu] compressing the ragged-rank workload (n=16384)")
    g1, _ = cauchy_hss(16384, tree.leaf_offsets(16384, 128), seed=1, tol=1e-10)
    cases.append(("c1 cauchy n=16384 m=128 ranks<=21", HSS.from_packed(g1), [1, 64], 64))
    g2 = inputs.synthetic_hss(tree.leaf_offsets(N, LEAF), RANK, seed=2)
    cases.append((f"c2 n={N} m={LEAF} k={RANK}", HSS.from_packed(g2), [1, 32], 1))
    kids = np.random.SeedSequence(3).spawn(512)[:32]
    batch = []
    for child in kids:
        rr = np.random.default_rng(child)
        n = 64 * int(rr.integers(32, 513))
        k = int(rr.choice([8, 16, 24]))
        batch.append(HSS.from_packed(inputs.synthetic_hss(tree.leaf_offsets(n, 64), k, seed=child)))
    rows = []
    for threads in (cores, 1):
        with threadpool_limits(limits=threads):
            for name, H, mm_r, sv_r in cases:
                for rr in mm_r:
                    X = inputs.rhs(H.n, rr, 5)
                    med, ts = _median_time(lambda: matvec(H, X), reps)
                    rows.append({"workload": name, "op": f"matmul r={rr}", "threads": threads,
                                 "median_s": round(med, 5), "runs_s": ts})
                    log(f"[cpu] {threads} thr {name} matmul r={rr}: {med:.4f} s")
                B = inputs.rhs(H.n, sv_r, 6)
                med, ts = _median_time(lambda: solve(H, B), reps)
                rows.append({"workload": name, "op": f"factor+solve r={sv_r}", "threads": threads,
                             "median_s": round(med, 5), "runs_s": ts})
                log(f"[cpu] {threads} thr {name} factor+solve r={sv_r}: {med:.4f} s")
            Bs = [inputs.rhs(H.n, 8, 7 + j) for j, H in enumerate(batch)]

            def run_batch():
                for H, B in zip(batch, Bs):
                    solve(H, B)
            med, ts = _median_time(run_batch, reps)
            rows.append({"workload": "c3 subset: 32 instances n=64*U{32..512} m=64 k in {8,16,24}",
                         "op": "factor+solve r=8 (all 32)", "threads": threads,
                         "median_s": round(med, 5), "runs_s": ts})
            log(f"[cpu] {threads} thr c3 subset: {med:.4f} s")
    out = {"metric": "FP64 oracle (unoptimized reference) wall time on the host",
           "host_cores": cores, "reps": reps, "warmup": 1, "timings": rows}
    _emit(out, args)


if __name__ == "__main__":
    main()
