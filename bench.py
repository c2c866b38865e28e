#!/usr/bin/env python3
"""Benchmark of the MM / PCG fused-lasso solver on one MI355X.

One step = one complete solve (every MM iteration: reweighting, the
tridiagonal factorization, the PCG inner loop with its X / X^T products,
Laplacian and preconditioner, the FP64 objective test) of the headline
workload with X, y and the edge set already resident in HBM.  Prints one
JSON line.

Workloads (--workload):
  c2  standard FLR, chain, n=1000, p=10000, X FP32 with AR(1) rho=0.5 rows,
      beta 50 blocks 80% zero, sigma=0.5, (lambda1, lambda2)=(0.5, 1.0), tol 1e-8
      (the configuration the headline metric is quoted on; default)
  c1  n=100, p=500, FP64 X (small case)
  c4  n=5000, p=50000, X stored BF16, y FP32
  c3  batched grid: two-dimensional FLR on the 100 x 100 lattice, n=2000,
      X FP32, the 16 x 16 log-spaced (lambda1, lambda2) grid over [0.01, 10]
      solved in one batched solve (FP64 matrix-core products X O and X^T U); a sample of
      the same columns through the plain single-solve path gives the plain
      solves/s beside it (a separate line, not the headline)
  c5  serving stream: Poisson arrivals of mixed requests (p in {1k, 5k, 10k,
      50k}, n = p/5, chain / lattice / all-pairs graphs, (lambda1, lambda2)
      log-uniform in [0.01, 10]) through the continuous-batching server, with
      HBM-footprint admission and warm starts; reports p50 / p99 latency and
      solves/s (a separate line, not the headline)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FLR solves/sec at p=10k + HBM GB/s; batched/mixed vs plain at 1e-6 obj gap"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # dense FP64 MFMA


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("flr_kernels.hip", "flr_internal.h", "flr_device.h"):
        with open(os.path.join(ROOT, "paper_1306_1970_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def make_workload(name):
    import flrgen

    if name == "c1":
        return flrgen.config1(), "c1_chain_n100_p500_f64"
    if name == "c4":
        return flrgen.config4(), "c4_chain_n5000_p50000_bf16"
    return flrgen.config2(), "c2_chain_ar1_n1000_p10000_f32"


def cpu_baseline(inst, gpu_cg_total: int, mm_sample: int):
    """The FP64 oracle (Algorithm 2, as it stands) on the same instance, on the
    host's cores.  mm_sample > 0: a bounded sample, the first mm_sample MM
    iterations, scaled to a whole solve by PCG steps (every PCG step of the
    oracle costs the same: two products with X, the Laplacian and two banded
    sweeps); mm_sample = 0: one complete solve, timed."""
    import oracle

    P = oracle.Problem.from_instance(inst)
    t0 = time.perf_counter()
    r = oracle.solve(P, inst.lam1, inst.lam2, eps=inst.eps, tol=inst.tol, max_iter=mm_sample, method=oracle.ALG2)
    dt = time.perf_counter() - t0
    if mm_sample <= 0:
        return {"value": 1.0 / dt, "unit": "solves/s", "cores": int(r.threads), "kind": "oracle",
                "sample": "one complete solve (%d MM iterations, %d PCG steps) in %.1f s on %d threads" % (
                    r.mm_iters, r.cg_iters, dt, r.threads)}
    cg = max(1, r.cg_iters)
    sec_per_solve = dt / cg * max(gpu_cg_total, 1)
    return {
        "value": 1.0 / sec_per_solve,
        "unit": "solves/s",
        "cores": int(r.threads),
        "kind": "oracle",
        "sample": "first %d MM iterations of the same solve (%d PCG steps, %.1f s) on %d threads, scaled by "
                  "PCG steps to the whole solve's %d" % (r.mm_iters, r.cg_iters, dt, r.threads, gpu_cg_total),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "paper"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--method", default="pcg", choices=["pcg", "cholesky"],
                    help="c1: Algorithm 2 (PCG) or Algorithm 1 (dense Cholesky per MM iteration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-mm-sample", type=int, default=60,
                    help="oracle baseline: MM iterations sampled (about 20 s on 16 host threads for c2)")
    ap.add_argument("--cpu-full", action="store_true", help="oracle baseline: one complete solve instead")
    ap.add_argument("--profile-reps", type=int, default=200)
    ap.add_argument("--mm-cap", type=int, default=0, help="cap on MM iterations (profiling runs only)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="after the solves, copy this many MiB with a plain device copy 3 times (reference "
                         "dispatches for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--grid-side", type=int, default=16, help="c3: lambda values per axis (side^2 columns)")
    ap.add_argument("--grid-tol", type=float, default=1e-7,
                    help="c3: relative objective change tolerance (1e-7 keeps the grid-vs-plain objective gap below 1e-6)")
    ap.add_argument("--plain-sample", type=int, default=2, help="c3: columns also solved by the plain path")
    ap.add_argument("--grid-max-iter", type=int, default=0, help="c3: cap on MM iterations (profiling runs only)")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=8.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-slots", type=int, default=4, help="concurrent solves (worker slots)")
    ap.add_argument("--serve-instances", type=int, default=1, help="resident problems per (p, graph) cell")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-ps", default="1000,5000,10000,50000")
    ap.add_argument("--paper-scenarios", default="C1,C2,C3,C4", help="paper: scenarios of sections 5.1/5.2")
    ap.add_argument("--paper-sizes", default="", help="paper: sizes to run (p, or q for C4); default all four")
    ap.add_argument("--paper-datasets", type=int, default=10, help="paper: data sets per scenario and size")
    ap.add_argument("--paper-first", type=int, default=0, help="paper: index of the first data set")
    ap.add_argument("--paper-inner", type=float, default=0.0, help="paper: inner tolerance (0: equal to 1e-5)")
    ap.add_argument("--serve-tol", type=float, default=1e-6)
    ap.add_argument("--serve-allpairs", default="pcg", choices=["pcg", "cholesky"],
                    help="c5: method for the all-pairs requests (PCG or Algorithm 1's dense Cholesky)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported (each GPU would take its own "
              "share of lambda columns or requests; nothing here spans GPUs)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1306_1970_amd as flr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "c5":
        return serve_main(args, flr)
    if args.workload == "c3":
        return grid_main(args, flr)
    if args.workload == "paper":
        return paper_main(args, flr)
    if args.method == "cholesky":
        return dense_main(args, flr)
    inst, wname = make_workload(args.workload)
    print("bench: workload %s n=%d p=%d m=%d dtype=%s" % (wname, inst.n, inst.p, inst.m, inst.dtype),
          file=sys.stderr, flush=True)
    ctx = flr.Context(0)
    prob = flr.Problem.from_instance(ctx, inst)
    prec = flr.FLR_PREC_FP64 if args.precision == "fp64" else flr.FLR_PREC_MIXED_FP32
    out = torch.zeros(inst.p, dtype=torch.float64, device="cuda:0")

    def one():
        return prob.solve(inst.lam1, inst.lam2, tol=inst.tol, out=out, precision=prec, max_iter=args.mm_cap)

    for _ in range(args.warmup):
        s = one()
        print("bench: warmup solve mm=%d cg=%d f=%.12g %.3fs" % (s.mm_iters, s.cg_iters, s.objective, s.seconds),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sols = []
    for _ in range(args.steps):
        sols.append(one())
        print("bench: solve mm=%d cg=%d f=%.12g %.3fs" % (sols[-1].mm_iters, sols[-1].cg_iters, sols[-1].objective,
                                                         sols[-1].seconds), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s = sols[-1]
    want = flr.FLR_ERR_MAX_ITER if args.mm_cap else flr.FLR_OK
    assert all(x.status in (flr.FLR_OK, want) for x in sols), [x.status for x in sols]

    # live per-kernel durations (HIP events on the problem's stream)
    a_us, b_us, c_us = flr.flr_profile_kernels(prob.h, args.profile_reps)
    xbytes = {0: 8, 1: 4, 2: 2}[inst.dtype]
    alg_bytes = inst.n * inst.p * xbytes + 8 * (inst.p + inst.n)  # X once + operand vector + result
    dom_name, dom_us = ("gemv_a", a_us) if a_us >= b_us else ("gemv_b", b_us)
    achieved = alg_bytes / (dom_us * 1e-6) / 1e9
    traffic = measured_traffic(dom_name, wname)
    # algorithmic bandwidth of the whole solve: per PCG step one pass over X (the one-pass bound of
    # X^T X p) plus about twelve p-vectors, the same per MM boundary, over the wall time of a solve
    step_bytes = inst.n * inst.p * xbytes + 12 * 8 * inst.p
    solve_gbs = (s.cg_iters + s.mm_iters) * step_bytes / (elapsed / args.steps) / 1e9

    line = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wname, "n": inst.n, "p": inst.p, "graph": inst.graph, "x_storage": {0: "f64", 1: "f32", 2: "bf16"}[inst.dtype],
                   "lambda1": inst.lam1, "lambda2": inst.lam2, "tol": inst.tol, "eps": inst.eps,
                   "precision": args.precision, "mm_iters": s.mm_iters, "cg_iters": s.cg_iters,
                   "objective": s.objective, "solve_effective_GBps": solve_gbs},
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "avg_us": dom_us,
                     "avg_us_how": "HIP events around %d back-to-back launches in the PCG-step state on the "
                                   "problem's stream" % args.profile_reps,
                     "algorithmic_bytes": alg_bytes, "other_kernel_us": b_us if dom_name == "gemv_a" else a_us,
                     "block_kernel_us": c_us, "solve_achieved": solve_gbs, "solve_frac": solve_gbs / HBM_PEAK_GBS},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(inst, s.cg_iters, 0 if args.cpu_full else args.cpu_mm_sample)
    if args.calibrate_copy:
        nb = args.calibrate_copy * (1 << 20)
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            evict = torch.full((nb // 4,), 2.0, dtype=torch.float32, device="cuda:0")  # pushes src out of the LLC
            del evict
            dst.copy_(src)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = nb
    prob.close()
    ctx.close()
    print(json.dumps(line), flush=True)


def dense_main(args, flr):
    """Algorithm 1 on the GPU: per MM iteration the dense system is assembled,
    factored by the blocked FP64 Cholesky on the matrix cores and solved."""
    import torch

    if args.workload != "c1":
        sys.exit("bench.py: --method cholesky runs on c1 (Algorithm 1 keeps dense p x p matrices; p <= 8192)")
    import oracle

    inst, wname = make_workload(args.workload)
    print("bench: workload %s n=%d p=%d m=%d (Algorithm 1)" % (wname, inst.n, inst.p, inst.m), file=sys.stderr,
          flush=True)
    ctx = flr.Context(0)
    prob = flr.Problem.from_instance(ctx, inst)
    out = torch.zeros(inst.p, dtype=torch.float64, device="cuda:0")

    def one():
        return prob.solve(inst.lam1, inst.lam2, tol=inst.tol, out=out, method=flr.FLR_METHOD_CHOLESKY,
                          max_iter=args.mm_cap)

    for _ in range(args.warmup):
        s = one()
        print("bench: warmup solve mm=%d f=%.12g %.3fs" % (s.mm_iters, s.objective, s.seconds), file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sols = []
    for _ in range(args.steps):
        sols.append(one())
        print("bench: solve mm=%d f=%.12g %.3fs" % (sols[-1].mm_iters, sols[-1].objective, sols[-1].seconds),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s = sols[-1]
    want = flr.FLR_ERR_MAX_ITER if args.mm_cap else flr.FLR_OK
    assert all(x.status in (flr.FLR_OK, want) for x in sols), [x.status for x in sols]
    asm_us, fac_us, sol_us = flr.flr_profile_dense(prob.h, inst.lam1, inst.lam2, args.profile_reps)
    fac_flops = inst.p ** 3 / 3.0  # Cholesky of the p x p system (the padding to 64 is not counted)
    achieved = fac_flops / (fac_us * 1e-6) / 1e12
    line = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wname, "method": "algorithm1_cholesky", "n": inst.n, "p": inst.p,
                   "graph": inst.graph, "x_storage": {0: "f64", 1: "f32", 2: "bf16"}[inst.dtype],
                   "lambda1": inst.lam1, "lambda2": inst.lam2, "tol": inst.tol, "eps": inst.eps,
                   "mm_iters": s.mm_iters, "objective": s.objective,
                   "ms_per_mm_iteration": 1000.0 * elapsed / args.steps / max(s.mm_iters, 1)},
        "roofline": {"bound": "mfma", "kernel": "cholesky_factor", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "avg_us": fac_us,
                     "avg_us_how": "HIP events around each of %d factorizations (%d launches each) on the "
                                   "problem's stream" % (args.profile_reps, 3 * ((inst.p + 63) // 64)),
                     "algorithmic_flops": fac_flops, "assembly_us": asm_us, "triangular_solves_us": sol_us},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        P = oracle.Problem.from_instance(inst)
        t0 = time.perf_counter()
        r = oracle.solve(P, inst.lam1, inst.lam2, eps=inst.eps, tol=inst.tol, method=oracle.ALG1)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 1.0 / dt, "unit": "solves/s", "cores": int(r.threads), "kind": "oracle",
                                "sample": "one complete Algorithm 1 solve (%d MM iterations) in %.1f s on %d threads"
                                          % (r.mm_iters, dt, r.threads)}
    prob.close()
    ctx.close()
    print(json.dumps(line), flush=True)


def paper_main(args, flr):
    """The paper's simulation scenarios (section 5.1: C1-C3 on a chain; 5.2:
    C4 on a lattice) at their sizes, ten data sets each, the four
    (lambda1, lambda2) settings, relative objective change 1e-5 and eps 1e-8,
    every solve from the method's own start.  Per cell: the mean and spread
    of the MM iteration counts and the GPU seconds per solve, beside the
    paper's MM and MMGPU columns (Tables C.1-C.4, other hardware: context)."""
    import numpy as np

    import flrgen

    printed = {(c["scenario"], c["size"], c["lambda1"], c["lambda2"]): c
               for c in json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables_c.json")))["cells"]}
    ctx = flr.Context(0)
    cells, t_all, n_all = [], 0.0, 0
    for sc in args.paper_scenarios.split(","):
        sizes = [int(x) for x in args.paper_sizes.split(",")] if args.paper_sizes else flrgen.PAPER_SIZES[sc]
        for size in sizes:
            rec = {lp: {"mm": [], "cg": [], "sec": [], "status": []} for lp in flrgen.PAPER_LAMBDAS}
            for d in range(args.paper_first, args.paper_first + args.paper_datasets):
                inst = flrgen.paper_scenario(sc, size, d)
                prob = flr.Problem.from_instance(ctx, inst)
                for lp in flrgen.PAPER_LAMBDAS:
                    t0 = time.perf_counter()
                    s = prob.solve(lp[0], lp[1], tol=flrgen.PAPER_TOL, eps=1e-8, inner_tol=args.paper_inner)
                    dt = time.perf_counter() - t0
                    r = rec[lp]
                    r["mm"].append(s.mm_iters)
                    r["cg"].append(s.cg_iters)
                    r["sec"].append(dt)
                    r["status"].append(s.status)
                    t_all += dt
                    n_all += 1
                prob.close()
                print("bench: %s size %d data set %d: MM %s" % (sc, size, d, [rec[lp]["mm"][-1] for lp in
                                                                              flrgen.PAPER_LAMBDAS]),
                      file=sys.stderr, flush=True)
            for lp in flrgen.PAPER_LAMBDAS:
                r, pc = rec[lp], printed.get((sc, size, lp[0], lp[1]), {})
                mm = np.array(r["mm"], dtype=float)
                cells.append({"scenario": sc, "size": size, "p": size * size if sc == "C4" else size,
                              "lambda1": lp[0], "lambda2": lp[1], "mm_mean": float(mm.mean()),
                              "mm_sd": float(mm.std(ddof=1)) if mm.size > 1 else 0.0,
                              "mm_min": int(mm.min()), "mm_max": int(mm.max()), "mm_all": [int(x) for x in mm],
                              "cg_mean": float(np.mean(r["cg"])), "gpu_seconds_mean": float(np.mean(r["sec"])),
                              "all_ok": all(x == flr.FLR_OK for x in r["status"]),
                              "paper_mm_iters": pc.get("mm_iters"), "paper_mm_seconds": pc.get("mm_seconds"),
                              "paper_mmgpu_iters": pc.get("mmgpu_iters"), "paper_mmgpu_seconds": pc.get("mmgpu_seconds")})
                c = cells[-1]
                print("bench: %s size %d lam (%g, %g): MM %.1f +- %.1f (paper MM %s), GPU %.4f s (paper MMGPU %s s, "
                      "MM %s s)" % (sc, size, lp[0], lp[1], c["mm_mean"], c["mm_sd"], c["paper_mm_iters"],
                                    c["gpu_seconds_mean"], c["paper_mmgpu_seconds"], c["paper_mm_seconds"]),
                      file=sys.stderr, flush=True)
    ctx.close()
    line = {
        "metric": "paper scenarios C1-C4 (sections 5.1, 5.2): MM iterations and GPU seconds per solve vs Tables C.1-C.4",
        "value": n_all / t_all,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": n_all,
        "warmup": 0,
        "ms_per_step": 1000.0 * t_all / n_all,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "paper_scenarios_%s" % args.paper_scenarios.replace(",", ""), "n": flrgen.PAPER_N,
                   "datasets": args.paper_datasets, "first_dataset": args.paper_first, "tol": flrgen.PAPER_TOL, "eps": 1e-8,
                   "inner_tol": args.paper_inner or flrgen.PAPER_TOL, "x_storage": "f64"},
        "cells": cells,
    }
    print(json.dumps(line), flush=True)


def grid_main(args, flr):
    """Batched lambda grid against the plain path on the same GPU."""
    import numpy as np

    import flrgen

    inst = flrgen.config3()
    vals = np.logspace(-2.0, 1.0, args.grid_side)
    l1, l2 = flrgen.grid_lambdas(vals)
    B = int(l1.size)
    print("bench: workload %s n=%d p=%d m=%d B=%d" % (inst.name, inst.n, inst.p, inst.m, B), file=sys.stderr,
          flush=True)
    os.environ.setdefault("FLR_PROGRESS", "1")
    ctx = flr.Context(0)
    prob = flr.Problem.from_instance(ctx, inst)
    # warm-up: one capped batched step prepares the FP64 copy of X, the
    # workspace for B columns and the GEMM handles
    prob.solve_grid(l1, l2, tol=1e-2, max_iter=1, max_cg=2)
    t0 = time.perf_counter()
    st, beta, res = prob.solve_grid(l1, l2, tol=args.grid_tol, max_iter=args.grid_max_iter)
    t_grid = time.perf_counter() - t0
    print("bench: grid of %d columns %.2f s, status %d, mm %d..%d, cg %d..%d" % (
        B, t_grid, st, min(r["mm_iters"] for r in res), max(r["mm_iters"] for r in res),
        min(r["cg_iters"] for r in res), max(r["cg_iters"] for r in res)), file=sys.stderr, flush=True)
    # plain path on a sample of the same columns (spread over the grid)
    pick = np.linspace(0, B - 1, args.plain_sample).round().astype(int) if args.plain_sample > 0 else []
    t_plain, gaps = 0.0, []
    for b in pick:
        t1 = time.perf_counter()
        s1 = prob.solve(l1[b], l2[b], tol=args.grid_tol)
        t_plain += time.perf_counter() - t1
        gaps.append(abs(s1.objective - res[b]["objective"]) / abs(s1.objective))
        print("bench: plain column %d lam=(%.3g,%.3g) %.2f s mm %d cg %d | grid mm %d cg %d | obj gap %.2e" % (
            b, l1[b], l2[b], time.perf_counter() - t1, s1.mm_iters, s1.cg_iters, res[b]["mm_iters"],
            res[b]["cg_iters"], gaps[-1]), file=sys.stderr, flush=True)
    plain_rate = len(pick) / t_plain if len(pick) else None
    grid_rate = B / t_grid
    ua, va = flr.flr_profile_grid(prob.h, B, 20)
    flops = 2.0 * inst.n * inst.p * B  # one GEMM
    dom_us = max(ua, va)
    achieved = flops / (dom_us * 1e-6) / 1e12
    prob.close()
    ctx.close()
    line = {
        "metric": "FLR batched lambda-grid solves/s vs plain path (same GPU)",
        "value": grid_rate,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": 1000.0 * t_grid,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c3_lattice_q100_n2000_f32_grid%dx%d" % (args.grid_side, args.grid_side),
                   "n": inst.n, "p": inst.p, "columns": B, "tol": args.grid_tol,
                   "plain_solves_per_s": plain_rate, "plain_sample_columns": [int(b) for b in pick],
                   "speedup_vs_plain": grid_rate / plain_rate if plain_rate else None,
                   "max_objective_gap_vs_plain": max(gaps) if gaps else None,
                   "status": int(st), "mm_iters_max": max(r["mm_iters"] for r in res),
                   "cg_iters_max": max(r["cg_iters"] for r in res)},
        "roofline": {"bound": "mfma", "kernel": "gemm_XO" if ua >= va else "gemm_XtU", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "avg_us": dom_us, "algorithmic_flops": flops, "other_kernel_us": min(ua, va)},
    }
    print(json.dumps(line), flush=True)


def serve_main(args, flr):
    """Serving stream: the arrivals are replayed in real time by a submitter
    thread; latency is submit-to-result as the server measures it."""
    import threading

    import numpy as np

    import flrgen

    ps = tuple(int(x) for x in args.serve_ps.split(","))
    reqs = flrgen.serving_requests(args.serve_requests, seed=5, rate=args.serve_rate, ps=ps)
    ctx = flr.Context(0)
    cells = {}
    t_setup = time.perf_counter()
    for r in reqs:
        key = (r["p"], r["graph"], r["slot"] % args.serve_instances)
        if key not in cells:
            inst = flrgen.serving_cell(r["p"], r["graph"], seed=1000 + len(cells))
            cells[key] = flr.Problem.from_instance(ctx, inst)
            print("bench: resident %s n=%d p=%d m=%d footprint %.1f MiB" % (inst.name, inst.n, inst.p, inst.m,
                  cells[key].footprint / 2 ** 20), file=sys.stderr, flush=True)
            del inst
    print("bench: %d resident problems in %.1f s" % (len(cells), time.perf_counter() - t_setup), file=sys.stderr,
          flush=True)
    budget = int(args.serve_budget_gib * 2 ** 30)
    srv = flr.flr_server_create(ctx.h, budget, args.serve_slots)
    opts = flr.default_opts(use_last=1)
    m_ap = flr.FLR_METHOD_CHOLESKY if args.serve_allpairs == "cholesky" else flr.FLR_METHOD_PCG
    opts_ap = flr.default_opts(use_last=1, method=m_ap)
    tickets = [None] * len(reqs)
    t0 = time.perf_counter()

    def submitter():
        for i, r in enumerate(reqs):
            wait = t0 + r["t"] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            h = cells[(r["p"], r["graph"], r["slot"] % args.serve_instances)].h
            o = opts_ap if r["graph"] == "allpairs" else opts
            tickets[i] = flr.flr_server_submit(srv, h, r["lam1"], r["lam2"], args.serve_tol, o)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    lat, mm, cg, status, by_graph = [], 0, 0, {}, {}
    for i, t in enumerate(tickets):
        st, res = flr.flr_server_poll(srv, t, True)
        lat.append(res.seconds)
        by_graph.setdefault(reqs[i]["graph"], []).append(res.seconds)
        mm += res.mm_iters
        cg += res.cg_iters
        status[st] = status.get(st, 0) + 1
        if (i + 1) % 16 == 0:
            print("bench: %d/%d done, %.1f s" % (i + 1, len(tickets), time.perf_counter() - t0), file=sys.stderr,
                  flush=True)
    elapsed = time.perf_counter() - t0
    flr.flr_server_destroy(srv)
    for p in cells.values():
        p.close()
    ctx.close()
    lat = np.array(lat)
    line = {
        "metric": "FLR serving: solves/s with p50/p99 latency (Poisson arrivals, mixed p and graphs)",
        "value": len(reqs) / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 0,
        "ms_per_step": 1000.0 * elapsed / len(reqs),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c5_serving_mixed_p%s" % "-".join(str(p) for p in ps), "requests": len(reqs),
                   "arrival_rate_per_s": args.serve_rate, "slots": args.serve_slots,
                   "resident_problems": len(cells), "budget_bytes": budget, "tol": args.serve_tol,
                   "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                   "max_s": float(lat.max()), "mm_iters": mm, "cg_iters": cg,
                   "allpairs_method": args.serve_allpairs,
                   "p50_s_by_graph": {g: float(np.percentile(v, 50)) for g, v in sorted(by_graph.items())},
                   "status_counts": {str(k): v for k, v in status.items()}},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
