#!/usr/bin/env python3
"""Benchmark of the FMM gravity forward model on one MI355X.

Workload (the metric's configuration): 64^3 cells on the unit cube, 2-point
Gauss rule per axis (2,097,152 source points), density = 32 seeded Gaussian
blobs + U[-0.01, 0.01] noise, g (3 components) at all 262,144 cell centres,
p = 10, mixed precision (FP32 P2P and FP32-MFMA M2L, FP64 expansions and
combine).  A step is one full grav_eval (P2M, M2M, M2L, L2L, P2P, L2P +
combine) with rho already resident in HBM.  The FP64 path is timed on the
same workload at the smallest p that reaches rel err <= 1e-6 (p = 12), and its
p = 10 error is reported beside it.

Prints ONE JSON line (rank 0).  Extra fields: pair-equivalent throughput,
p50/p99 step latency, relative L2 error against the FP64 oracle on a seeded
sample of targets, the dominant kernel's roofline, the oracle's CPU
throughput on that sample, and the FP64 result.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "gz evals/s (src·tgt pairs/s equiv) at rel err ≤1e-6/1e-4; p50/p99 latency"
PEAK = {"fp64_mfma": 78.6, "fp32_mfma": 157.3, "fp32_vector": 157.3, "fp64_vector": 78.6}
P2P_FLOP_PER_PAIR = 20.0  # Sec. 1.1 cost model: 5 add + 7 mul + 1 sqrt ~ 20 multiplications


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--p", type=int, default=10)
    ap.add_argument("--p64", type=int, default=12)
    ap.add_argument("--leaf", type=int, default=512)
    ap.add_argument("--sample", type=int, default=2048, help="oracle targets for cpu_baseline/rel_err")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--no-direct", action="store_true", help="skip the GPU direct-sum comparison")
    ap.add_argument("--serve", type=int, default=0, metavar="COUNT",
                    help="only run the serving workload: COUNT Poisson requests (rate 50/s, n in [32, 192])")
    ap.add_argument("--paper-sequence", action="store_true",
                    help="only time the FMM on the paper's model over its mesh sequence (Mbar = 12 .. 384)")
    ap.add_argument("--crossover", action="store_true",
                    help="only time FMM vs GPU direct sum over station counts (summation/FMM crossover)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (HBM counter calibration)")
    return ap.parse_args()


def timed_steps(plan, rho, out, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.eval(rho, out)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(steps):
        plan.eval(rho, out)
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    total_ms = evs[0].elapsed_time(evs[steps])
    return total_ms, lat, wall


def stage_profile(plan, rho, out, steps):
    """Average per-stage duration (HIP events on the eval stream)."""
    import torch
    plan.set_profiling(True)
    acc = {}
    for _ in range(steps):
        plan.eval(rho, out)
        for name, ms in plan.stage_times():
            acc[name] = acc.get(name, 0.0) + ms
    plan.set_profiling(False)
    torch.cuda.synchronize()
    return {k: v / steps for k, v in acc.items()}


def measured_traffic(kernel_name):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None if it is for another kernel or the kernel sources have
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "m2l_volume64_q2_hbm_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    src = b"".join(open(os.path.join(ROOT, "paper_1107_5951_amd", "csrc", f), "rb").read()
                   for f in ("m2l.hip", "eval_common.hpp"))
    if fields.get("source_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
        return None
    if not kernel_name.startswith(fields.get("kernel", "?")):
        return None
    return float(fields["traffic_bytes_per_launch"])


def pct(xs, q):
    s = sorted(xs)
    return s[min(len(s) - 1, int(round(q / 100.0 * (len(s) - 1))))]


def paper_sequence(args):
    """The paper's model (Sec. 3) on Mbar^3 meshes, 1-point rule, gz at every
    cell centroid, p = 8, 27 cells per leaf (the setting of its FMM timing
    table), FP64 and mixed precision: plan time and evaluation time."""
    import torch

    import paper_1107_5951_amd as G
    import workloads as W
    rows = []
    for nbar in (12, 24, 48, 96, 192, 384):
        grid, rho_h = W.paper_model(nbar)
        rho = torch.as_tensor(rho_h, device="cuda")
        del rho_h
        row = {"Mbar": nbar, "cells": nbar ** 3}
        for prec, tag in ((G.GRAV_FP64, "fp64"), (G.GRAV_MIXED, "mixed")):
            t0 = time.perf_counter()
            plan = G.Plan(G.PlanSpec(n=(nbar, nbar, nbar), h=grid.h, origin=grid.origin, quad_order=1,
                                     voxel_centres=True, components=1, p=8, leaf_size=27, precision=prec,
                                     G=W.G_SI))
            plan_s = time.perf_counter() - t0
            out = torch.empty(plan.out_shape, dtype=torch.float64, device="cuda")
            plan.eval(rho, out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                plan.eval(rho, out)
            e1.record()
            torch.cuda.synchronize()
            row[tag] = {"plan_s": plan_s, "eval_ms": e0.elapsed_time(e1) / 5, "levels": plan.levels}
            del plan, out
        rows.append(row)
        print(json.dumps(row), flush=True)
        del rho
        torch.cuda.empty_cache()
    print(json.dumps({"paper_sequence": rows}), flush=True)


def serving(args):
    """Many small forward solves: a seeded Poisson trace (rate 50/s) of
    meshes n = round(exp U[ln 32, ln 192]), q in {1, 2}, gz at n x n
    stations, p = 8 mixed.  Plans are built first (timed separately); then
    the trace is served back to back (capacity) and at its arrival times
    (latency under load)."""
    import torch

    from paper_1107_5951_amd import serve
    reqs = serve.poisson_trace(args.serve, rate=50.0, seed=1005, host_blobs=False)
    srv = serve.GravServer(n_streams=4)
    t0 = time.perf_counter()
    for r in reqs:
        srv.cache.get(r.n, r.q)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    _, cap = srv.run(reqs)
    _, live = srv.run(reqs, realtime=True)
    srv.close()
    print(json.dumps({"workload": "serving: %d Poisson requests at 50/s, n in [32, 192], q in {1, 2}, "
                                  "gz at n^2 stations, p=8 mixed, forward only" % args.serve,
                      "plans": len(set((r.n, r.q) for r in reqs)), "plan_build_s": build_s,
                      "capacity": cap, "realtime": live}), flush=True)


def crossover(args):
    """Summation vs FMM as the number of stations grows (cf. the paper's
    crossover discussion, Sec. 4): a fixed 64^3 mesh, 1-point rule, gz at
    ns x ns stations at z = 1.1, mixed precision p = 8; the summation by the
    1-point rule (SUM-G1, grav_direct) and in closed form (SUM-AN,
    grav_analytic, FP64)."""
    import torch

    import paper_1107_5951_amd as G
    import workloads as W
    n = 64
    grid = W.Grid.unit(n)
    rho = torch.as_tensor(W.gaussian_blobs(grid, 32, 1002), device="cuda")
    rows = []
    for ns in (2, 4, 8, 16, 32, 64, 128, 256):
        plan = G.Plan(G.PlanSpec(n=(n, n, n), h=grid.h, points=W.stations(ns, 1.1), components=1, p=8,
                                 leaf_size=64, precision=G.GRAV_MIXED))
        out = torch.empty(plan.out_shape, dtype=torch.float64, device="cuda")
        t = {}
        for name, fn in (("fmm", plan.eval), ("direct", plan.direct), ("analytic", plan.analytic)):
            fn(rho, out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10 if name == "fmm" else 3
            e0.record()
            for _ in range(reps):
                fn(rho, out)
            e1.record()
            torch.cuda.synchronize()
            t[name] = e0.elapsed_time(e1) / reps
        rows.append({"stations": ns * ns, "fmm_ms": t["fmm"], "direct_ms": t["direct"],
                     "analytic_ms": t["analytic"]})
        print(json.dumps(rows[-1]), flush=True)
    faster = [r["stations"] for r in rows if r["fmm_ms"] < r["direct_ms"]]
    faster_an = [r["stations"] for r in rows if r["fmm_ms"] < r["analytic_ms"]]
    print(json.dumps({"crossover_stations": min(faster) if faster else None,
                      "crossover_stations_analytic": min(faster_an) if faster_an else None,
                      "mesh": "64^3, q=1", "rows": rows}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8, "copies": 3}))
        return

    import paper_1107_5951_amd as G
    import workloads as W

    if args.crossover:
        crossover(args)
        return
    if args.serve:
        serving(args)
        return
    if args.paper_sequence:
        paper_sequence(args)
        return

    n = args.n
    grid = W.Grid.unit(n)
    rho_h = W.gaussian_blobs(grid, 32, 1002, noise=0.01)
    rho = torch.as_tensor(rho_h, device="cuda")
    M = grid.ncell

    def make(prec, p):
        t0 = time.perf_counter()
        plan = G.Plan(G.PlanSpec(n=(n, n, n), h=grid.h, quad_order=2, voxel_centres=True,
                                 components=3, p=p, leaf_size=args.leaf, precision=prec))
        return plan, time.perf_counter() - t0

    plan, plan_s = make(G.GRAV_MIXED, args.p)
    out = torch.empty(plan.out_shape, dtype=torch.float64, device="cuda")
    total_ms, lat, wall = timed_steps(plan, rho, out, args.steps, args.warmup)
    ms = total_ms / args.steps
    stages = stage_profile(plan, rho, out, max(5, min(args.steps, 20)))
    m2l_pairs, p2p_pairs, n_src = plan.work()
    g_mixed = out[0].cpu().numpy()

    value = M / (ms * 1e-3)
    P2 = args.p * args.p
    # dominant kernel and its roofline (algorithmic flops per launch / stage time)
    b = plan.leaf_cells
    n_leaf_src = (-(-n // b)) ** 3
    flops_m2l = 2.0 * P2 * P2 * m2l_pairs
    flops_p2p = P2P_FLOP_PER_PAIR * p2p_pairs
    flops_near = 27 * 2.0 * (4 * b ** 3) * b ** 3 * n_leaf_src
    cand = {
        "m2l": (flops_m2l, "k_m2l<%d,%d,2,float> (M2L, FP32 MFMA 16x16x4)" % (-(-P2 // 16), -(-P2 // 4)), "mfma",
                "fp32_mfma"),
        "near_lat": (flops_near, "k_near_lat<4,2,float> (lattice near field, FP32 MFMA 16x16x4)", "mfma",
                     "fp32_mfma"),
        "p2p": (flops_p2p, "k_p2p<float> (direct near field, FP32 VALU)", "alu", "fp32_vector"),
    }
    dom = max((k for k in cand if k in stages), key=lambda k: stages[k])
    fl, kname, bound, pk = cand[dom]
    roof = {"kernel": kname, "bound": bound, "achieved": fl / (stages[dom] * 1e-3) / 1e12,
            "peak": PEAK[pk], "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(kname)
    roof["kernel_ms"] = stages.get(dom)

    res = {
        "metric": METRIC, "value": value, "unit": "gz evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (mixed: M2L and lattice near field on FP32 MFMA; expansions, M2M/L2L/L2P and combine in f64)",
        "data": "synthetic",
        "config": {"workload": "%d^3 cells, 2-point Gauss (%d sources), g at %d cell centres, p=%d, "
                               "mixed precision, leaf %d cells" % (n, n_src, M, args.p, plan.leaf_cells ** 3),
                   "levels": plan.levels, "leaf_cells": plan.leaf_cells, "batch": 1},
        "pair_equiv_per_s": value * n_src,
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
        "plan_s": plan_s,
        "stages_ms": stages,
        "work": {"m2l_box_pairs": m2l_pairs, "p2p_point_pairs": p2p_pairs, "m2l_gflop": flops_m2l / 1e9,
                 "near_lat_gflop": flops_near / 1e9 if "near_lat" in stages else None,
                 "p2p_gflop_20": flops_p2p / 1e9},
        "roofline": roof,
    }

    fp64 = None
    if not args.no_fp64:
        del plan
        plan64, plan64_s = make(G.GRAV_FP64, args.p64)
        tms, lat64, _ = timed_steps(plan64, rho, out, args.steps, args.warmup)
        st64 = stage_profile(plan64, rho, out, 5)
        g64 = out[0].cpu().numpy()
        ms64 = tms / args.steps
        m2l64, _, _ = plan64.work()
        del plan64
        fp64 = {"p": args.p64, "value": M / (ms64 * 1e-3), "ms_per_step": ms64,
                "p50_ms": pct(lat64, 50), "p99_ms": pct(lat64, 99), "stages_ms": st64,
                "m2l_tflops": 2.0 * args.p64 ** 4 * m2l64 / (st64.get("m2l", 1e9) * 1e-3) / 1e12}
        plan10, _ = make(G.GRAV_FP64, args.p)
        plan10.eval(rho, out)
        torch.cuda.synchronize()
        g64_p = out[0].cpu().numpy()
        del plan10
        res["fp64"] = fp64

    if not args.no_direct:
        # the summation method on the same GPU, same targets and arithmetic
        # class (FP32 pairs for the mixed plan): one evaluation
        plan_d, _ = make(G.GRAV_MIXED, args.p)
        plan_d.direct(rho, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        plan_d.direct(rho, out)
        ev1.record()
        torch.cuda.synchronize()
        dms = ev0.elapsed_time(ev1)
        g_direct = out[0].cpu().numpy()
        del plan_d
        res["direct_sum"] = {"ms": dms, "value": M / (dms * 1e-3), "pairs_per_s": M * n_src / (dms * 1e-3),
                             "fmm_speedup": dms / ms, "kernel": "k_direct<float> (Sec. 2.1 summation, FP32)"}

    if not args.no_cpu:
        import oracle
        idx = W.sample_indices(M, args.sample, seed=7)
        tg = grid.centres()[idx]
        threads = oracle.num_threads()
        t0 = time.perf_counter()
        ref = oracle.forward(rho_h, grid.origin, grid.h, 2, tg, comps=3)
        cpu_s = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": len(idx) / cpu_s, "unit": "gz evals/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "%d seeded cell-centre targets (of %d) x all %d source points, "
                                         "FP64 direct sum, %.1f s" % (len(idx), M, n_src, cpu_s),
                               "pair_equiv_per_s": len(idx) * n_src / cpu_s}
        res["rel_err"] = oracle.rel_l2(g_mixed[idx], ref)
        if "direct_sum" in res:
            res["direct_sum"]["rel_err"] = oracle.rel_l2(g_direct[idx], ref)
        res["rel_err_bar"] = 1e-4
        if fp64 is not None:
            fp64["rel_err"] = oracle.rel_l2(g64[idx], ref)
            fp64["rel_err_p%d" % args.p] = oracle.rel_l2(g64_p[idx], ref)
            fp64["rel_err_bar"] = 1e-6
    line = json.dumps(res)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
