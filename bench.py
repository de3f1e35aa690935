#!/usr/bin/env python3
"""Benchmark of the FMM gravity forward model on one MI355X.

Headline workload: 256^3 cells on the unit cube (16,777,216 cells), 1-point
rule (one source point per cell), density = 64 seeded Gaussian blobs plus the
constant-density prism [0.4, 0.6]^2 x [0.2, 0.5] (rho = 1), g (3 components)
at 512 x 512 stations at z = 1.1 and at every cell centre (17,039,360
targets), mixed precision, leaf edge 4 cells.  The expansion order is p = 10,
the smallest order at which the mixed-precision solve meets rel err <= 1e-4
both against the FP64 oracle on 4096 seeded targets and, for the prism alone,
against its closed form; the workload's nominal p = 8 is timed beside it with
its errors.  A step is one full grav_eval (P2M, M2M, M2L, L2L, lattice near
field, P2P, L2P + combine) with rho already resident in HBM.  The FP64 solve
of the same workload runs at p = 16, the smallest order meeting 1e-6 on both
checks.

Also reported (extra fields): the 64^3-cell, 2-point-rule volume workload
(mixed p = 10 and FP64 p = 12), and the batched workload of 32 density
models on one 128^3-cell tree with gz at 256 x 256 stations (mixed p = 10
against FP64 p = 14, batched and as 32 single-model solves).

Prints ONE JSON line.  Extra fields: pair-equivalent throughput, p50/p99 step
latency, relative L2 error against the FP64 oracle on seeded targets, the
dominant kernel's roofline, the oracle's CPU throughput (all cores and one
thread).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "gz evals/s (src·tgt pairs/s equiv) at rel err ≤1e-6/1e-4; p50/p99 latency"
PEAK = {"fp64_mfma": 78.6, "fp32_mfma": 157.3, "fp32_vector": 157.3, "fp64_vector": 78.6, "hbm": 8000.0}
P2P_FLOP_PER_PAIR = 20.0  # Sec. 1.1 cost model: one kernel evaluation ~ 20 flops
PRISM = ((0.4, 0.6), (0.4, 0.6), (0.2, 0.5))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="cells per axis of the headline mesh")
    ap.add_argument("--p", type=int, default=10, help="expansion order of the headline (mixed) solve")
    ap.add_argument("--p-nominal", type=int, default=8, help="the workload's nominal order, timed beside it")
    ap.add_argument("--p64", type=int, default=16, help="expansion order of the FP64 solve")
    ap.add_argument("--sample", type=int, default=4096, help="seeded oracle targets for rel_err")
    ap.add_argument("--cpu-one-thread", type=int, default=32,
                    help="targets of the one-thread oracle timing")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline only (no 64^3 or batched rows)")
    ap.add_argument("--timed-only", action="store_true",
                    help="only the headline's timed evaluations (one plan; for kernel profiles)")
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    ap.add_argument("--serve", type=int, default=0, metavar="COUNT",
                    help="only run the serving workload: COUNT Poisson requests (rate 50/s, n in [32, 192])")
    ap.add_argument("--paper-sequence", action="store_true",
                    help="only time the FMM on the paper's model over its mesh sequence (Mbar = 12 .. 384)")
    ap.add_argument("--crossover", action="store_true",
                    help="only time FMM vs GPU direct sum over station counts (summation/FMM crossover)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 128^3 x 32-model batched forward and adjoint rows (for kernel profiles)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 3 device-to-device copies of MIB MiB (HBM counter calibration)")
    return ap.parse_args()


def say(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def timed_steps(plan, rho, out, steps, warmup):
    """Wall time of `steps` evaluations on the current stream (HIP events),
    after `warmup` untimed ones; per-step latencies for p50/p99."""
    import torch
    for _ in range(warmup):
        plan.eval(rho, out)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record()
    for i in range(steps):
        plan.eval(rho, out)
        evs[i + 1].record()
    torch.cuda.synchronize()
    lat = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    return evs[0].elapsed_time(evs[steps]) / steps, lat


def stage_profile(plan, rho, out, steps):
    """Average per-stage duration: HIP events recorded by the library on the
    evaluation stream around each stage's launches."""
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


def adjoint_profile(plan, out_shape, reps):
    """Time of the adjoint (grav_adjoint) on a seeded residual, HIP events
    on the current stream, and its per-stage durations."""
    import torch
    res = torch.randn(out_shape, dtype=torch.float64, device="cuda",
                      generator=torch.Generator(device="cuda").manual_seed(1004))
    drho = torch.empty(plan.rho_shape, dtype=torch.float64, device="cuda")
    plan.adjoint(res, drho)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.adjoint(res, drho)
    e1.record()
    torch.cuda.synchronize()
    plan.set_profiling(True)
    acc = {}
    for _ in range(reps):
        plan.adjoint(res, drho)
        for name, ms in plan.stage_times():
            acc[name] = acc.get(name, 0.0) + ms
    plan.set_profiling(False)
    torch.cuda.synchronize()
    del res, drho
    return e0.elapsed_time(e1) / reps, {k: v / reps for k, v in acc.items()}


def measured_traffic(profile, kernel_name):
    """HBM bytes per launch of the dominant kernel from a committed counter
    summary under profiles/, or None if it covers another kernel or the
    kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
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
                   for f in ("m2l.hip", "eval_common.hpp", "internal.hpp", "resolve.hpp"))
    if fields.get("source_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
        return None
    if not kernel_name.startswith(fields.get("kernel", "?")):
        return None
    return float(fields["traffic_bytes_per_launch"])


def pct(xs, q):
    s = sorted(xs)
    return s[min(len(s) - 1, int(round(q / 100.0 * (len(s) - 1))))]


# mixed plans at these orders run the M2L once per reflection orbit of
# offsets (k_m2l_orb): the eight sign classes of the coefficients hold at
# most 16 each up to p = 10, and below p = 10 the per-offset kernel is as
# fast or faster.  (Plans whose orbits hold few offsets with a source, such
# as stations above the source block, keep the per-offset kernel; in the
# rows below their roofline stage is not the M2L.)
M2L_ORBIT_ORDERS = (10,)


def m2l_orbit(p, prec):
    from paper_1107_5951_amd import GRAV_FP64
    return prec != GRAV_FP64 and p in M2L_ORBIT_ORDERS


def m2l_kernel_name(p, prec):
    from paper_1107_5951_amd import GRAV_FP64
    p2 = p * p
    if prec == GRAV_FP64:
        return "k_m2l<%d,%d,*,double,*>" % (-(-p2 // 16), -(-p2 // 4))
    if m2l_orbit(p, prec):
        return "k_m2l_orb<*>"
    return "k_m2l<%d,%d,*,float,*>" % (-(-p2 // 16), -(-p2 // 4))


def m2l_label(p, prec):
    from paper_1107_5951_amd import GRAV_FP64
    f64 = prec == GRAV_FP64
    if m2l_orbit(p, prec):
        return m2l_kernel_name(p, prec) + (" (M2L per reflection orbit of offsets, FP32 MFMA 16x16x4; work"
                                           " counted as the per-offset product, 2 p^4 per box pair)")
    return m2l_kernel_name(p, prec) + " (M2L, %s MFMA 16x16x4%s)" % (
        "FP64" if f64 else "FP32", "" if f64 or not 0 < p * p % 16 <= 4 else ", the last row block 4x4x1")


def roofline(plan, stages, p, prec, profile):
    """Roofline of the dominant stage: its algorithmic work per launch over
    the stage's event-measured duration.  Compute-bound stages count flops
    (M2L: 2 p^4 per box pair and model; lattice near field: 27 x 2 x C b^3 x
    b^3 per leaf and model for C output components; M2M: 8 x 2 p^4 per parent box and model); the P2M
    on a surface-target plan is bound by HBM and counts the bytes it must
    move (the densities read and the leaf expansions written)."""
    from paper_1107_5951_amd import GRAV_FP64
    m2l_pairs, p2p_pairs, _ = plan.work()
    B = plan.spec.batch
    b = plan.leaf_cells
    n = [int(v) for v in plan.spec.n]
    L = plan.levels
    leaves = [-(-v // b) for v in n]
    n_leaf_src = leaves[0] * leaves[1] * leaves[2]
    parents = 0
    for lvl in range(2, L):
        c = 1
        for a in range(3):
            c *= -(-leaves[a] // (1 << (L - lvl)))
        parents += c
    f64 = prec == GRAV_FP64
    mm = "fp64_mfma" if f64 else "fp32_mfma"
    ps = -(-p * p // 16) * 16
    cand = {
        "m2l": (2.0 * p ** 4 * m2l_pairs * B, m2l_label(p, prec), "mfma", mm, "TFLOP/s"),
        "near_lat": (27 * 2.0 * (plan.spec.components * b ** 3) * b ** 3 * n_leaf_src * B,
                     "k_near_lat<%d,2,%s> (lattice near field, %s MFMA 16x16x4)"
                     % ((2, "double", "FP64") if f64 else (4, "float", "FP32")), "mfma", mm, "TFLOP/s"),
        "m2m": (8 * 2.0 * p ** 4 * parents * B, "k_m2m_lds<%d> / k_m2m_split<%d> (M2M, FP64 MFMA 16x16x4)"
                % (ps // 16, ps // 16), "mfma", "fp64_mfma", "TFLOP/s"),
        # the leaf's cells times the lattice P2M matrix (p^2 x b^3, FP64)
        "p2m": (2.0 * p * p * b ** 3 * n_leaf_src * B, "k_p2m_mfma<%d> (P2M, FP64 MFMA 16x16x4)" % (ps // 16),
                "mfma", "fp64_mfma", "TFLOP/s"),
    }
    if "near_lat" not in stages:
        # every near pair is a direct (point) pair only without the lattice path
        cand["p2p"] = (P2P_FLOP_PER_PAIR * p2p_pairs * B, "k_p2p (direct near field, VALU)", "alu",
                       "fp64_vector" if f64 else "fp32_vector", "TFLOP/s")
    live = [k for k in cand if k in stages and cand[k][0] > 0]
    dom = max(live, key=lambda k: stages[k])
    work, kname, bound, pk, unit = cand[dom]
    scale = 1e9 if unit == "GB/s" else 1e12
    roof = {"kernel": kname, "bound": bound, "achieved": work / (stages[dom] * 1e-3) / scale,
            "peak": PEAK[pk], "unit": unit}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(profile, kname) if profile else None
    roof["kernel_ms"] = stages.get(dom)
    roof["work_per_launch"] = work
    return roof


def sample_targets(st, grid, idx):
    """Positions of the evaluation points idx of a plan whose points are the
    stations st followed by every cell centre (x fastest)."""
    import numpy as np
    ns = st.shape[0]
    out = np.empty((idx.size, 3))
    sel = idx < ns
    out[sel] = st[idx[sel]]
    c = idx[~sel] - ns
    ix, iy, iz = c % grid.nx, (c // grid.nx) % grid.ny, c // (grid.nx * grid.ny)
    out[~sel] = np.stack([grid.origin[0] + (ix + 0.5) * grid.h, grid.origin[1] + (iy + 0.5) * grid.h,
                          grid.origin[2] + (iz + 0.5) * grid.h], axis=1)
    return out


def gather_rows(out, idx):
    import torch
    return out[0].index_select(0, torch.as_tensor(idx, device=out.device)).cpu().numpy()


# ----------------------------------------------------------------------------
def headline(args):
    import numpy as np
    import torch

    import paper_1107_5951_amd as G
    import workloads as W

    n = args.n
    grid = W.Grid.unit(n)
    st = W.stations(512, 1.1)
    rho_h = W.gaussian_blobs(grid, 64, 1003) + W.box_density(grid, PRISM, 1.0)
    rho = torch.as_tensor(rho_h, device="cuda")
    M = st.shape[0] + grid.ncell
    idx = W.sample_indices(M, args.sample, seed=7)

    def make(prec, p, points=st, centres=True):
        t0 = time.perf_counter()
        plan = G.Plan(G.PlanSpec(n=(n, n, n), h=grid.h, quad_order=1, points=points, voxel_centres=centres,
                                 components=3, p=p, leaf_size=64, precision=prec))
        return plan, time.perf_counter() - t0

    say("headline plan: %d^3 cells, %d targets, mixed p=%d" % (n, M, args.p))
    plan, plan_s = make(G.GRAV_MIXED, args.p)
    out = torch.empty(plan.out_shape, dtype=torch.float64, device="cuda")
    ms, lat = timed_steps(plan, rho, out, args.steps, args.warmup)
    stages = stage_profile(plan, rho, out, max(5, min(args.steps, 20)))
    m2l_pairs, p2p_pairs, n_src = plan.work()
    g_sample = gather_rows(out, idx)
    roof = roofline(plan, stages, args.p, G.GRAV_MIXED, "m2l_volume256_q1_hbm_traffic.md")
    adj_ms, adj_stages = (None, None) if args.timed_only else adjoint_profile(plan, plan.out_shape, 5)
    levels, leaf = plan.levels, plan.leaf_cells
    resident, per_call = plan.bytes()
    del plan
    value = M / (ms * 1e-3)
    res = {
        "metric": METRIC, "value": value, "unit": "gz evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (mixed: M2L and lattice near field on FP32 MFMA; expansions, M2M/L2L/L2P and combine in f64)",
        "data": "synthetic",
        "config": {"workload": "%d^3 cells, 1-point rule (%d sources), 64 seeded blobs + prism, g at %d x %d "
                               "stations (z=1.1) + all %d cell centres (%d targets), p=%d, mixed precision, "
                               "leaf %d cells" % (n, n_src, 512, 512, grid.ncell, M, args.p, leaf ** 3),
                   "levels": levels, "leaf_cells": leaf, "batch": 1, "p": args.p, "p_nominal": args.p_nominal},
        "pair_equiv_per_s": value * n_src,
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
        "plan_s": plan_s, "plan_bytes": {"resident": resident, "per_call": per_call},
        "stages_ms": stages,
        "work": {"m2l_box_pairs": m2l_pairs, "p2p_point_pairs": p2p_pairs,
                 "m2l_gflop": 2.0 * args.p ** 4 * m2l_pairs / 1e9},
        "roofline": roof,
        "adjoint": {"ms": adj_ms, "stages_ms": adj_stages,
                    "what": "grad of 0.5||g - d||^2 w.r.t. rho (grav_adjoint, exact transpose) at the same plan"},
    }

    if args.timed_only:
        return res
    # the prism alone at the stations (checked against its closed form in
    # the oracle leg below)
    say("prism alone at the stations")
    rho_p = torch.as_tensor(W.box_density(grid, PRISM, 1.0), device="cuda")
    prism_gz = {}
    for prec, p in ((G.GRAV_MIXED, args.p), (G.GRAV_MIXED, args.p_nominal)) + (
            () if args.no_fp64 else ((G.GRAV_FP64, args.p64),)):
        pl, _ = make(prec, p, centres=False)
        prism_gz["%s_p%d" % ("fp64" if prec == G.GRAV_FP64 else "mixed", p)] = pl.eval(rho_p)[:, 2].cpu().numpy()
        del pl
    del rho_p

    say("nominal order p=%d" % args.p_nominal)
    plan8, _ = make(G.GRAV_MIXED, args.p_nominal)
    ms8, lat8 = timed_steps(plan8, rho, out, max(5, args.steps // 2), 2)
    st8 = stage_profile(plan8, rho, out, 3)
    g8 = gather_rows(out, idx)
    res["nominal_p"] = {"p": args.p_nominal, "value": M / (ms8 * 1e-3), "ms_per_step": ms8,
                        "p50_ms": pct(lat8, 50), "p99_ms": pct(lat8, 99), "stages_ms": st8,
                        "roofline": roofline(plan8, st8, args.p_nominal, G.GRAV_MIXED, None)}
    del plan8

    g64 = None
    if not args.no_fp64:
        say("fp64 p=%d" % args.p64)
        plan64, p64_s = make(G.GRAV_FP64, args.p64)
        ms64, lat64 = timed_steps(plan64, rho, out, 3, 1)
        st64 = stage_profile(plan64, rho, out, 2)
        g64 = gather_rows(out, idx)
        res["fp64"] = {"p": args.p64, "value": M / (ms64 * 1e-3), "ms_per_step": ms64,
                       "p50_ms": pct(lat64, 50), "p99_ms": pct(lat64, 99), "plan_s": p64_s, "stages_ms": st64,
                       "roofline": roofline(plan64, st64, args.p64, G.GRAV_FP64, None),
                       "mixed_speedup": ms64 / ms}
        del plan64
    del out
    torch.cuda.empty_cache()

    if not args.no_cpu:
        import oracle
        tg = sample_targets(st, grid, idx)
        threads = oracle.num_threads()
        say("oracle on %d targets x %d sources, %d threads" % (len(idx), n_src, threads))
        t0 = time.perf_counter()
        ref = oracle.forward(rho_h, grid.origin, grid.h, 1, tg, comps=3)
        cpu_s = time.perf_counter() - t0
        k1 = min(args.cpu_one_thread, len(idx))
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.forward(rho_h, grid.origin, grid.h, 1, tg[:k1], comps=3)
        cpu1_s = time.perf_counter() - t0
        oracle.set_threads(threads)
        res["cpu_baseline"] = {
            "value": len(idx) / cpu_s, "unit": "gz evals/s", "cores": threads, "kind": "oracle",
            "sample": "%d seeded targets (of %d: stations and cell centres) x all %d source points, FP64 "
                      "direct sum, %.1f s" % (len(idx), M, n_src, cpu_s),
            "pair_equiv_per_s": len(idx) * n_src / cpu_s,
            "one_thread": {"value": k1 / cpu1_s, "unit": "gz evals/s", "cores": 1,
                           "sample": "first %d of the same targets, %.1f s" % (k1, cpu1_s),
                           "pair_equiv_per_s": k1 * n_src / cpu1_s}}
        from oracle import prism
        exact = prism.prism_gz(st, W.snapped_box(grid, PRISM), 1.0, 1.0)
        res["prism_vs_closed_form"] = {k: float(np.linalg.norm(v - exact) / np.linalg.norm(exact))
                                       for k, v in prism_gz.items()}
        res["rel_err"] = oracle.rel_l2(g_sample, ref)
        res["rel_err_bar"] = 1e-4
        res["rel_err_targets"] = len(idx)
        res["nominal_p"]["rel_err"] = oracle.rel_l2(g8, ref)
        if g64 is not None:
            res["fp64"]["rel_err"] = oracle.rel_l2(g64, ref)
            res["fp64"]["rel_err_bar"] = 1e-6
    return res


def volume64(args):
    """64^3 cells, 2-point rule (2,097,152 sources), 32 blobs + noise, g at
    all 262,144 cell centres: mixed p = 10 and FP64 p = 12."""
    import torch

    import paper_1107_5951_amd as G
    import workloads as W
    n = 64
    grid = W.Grid.unit(n)
    rho_h = W.gaussian_blobs(grid, 32, 1002, noise=0.01)
    rho = torch.as_tensor(rho_h, device="cuda")
    M = grid.ncell
    idx = W.sample_indices(M, args.sample, seed=7)
    row = {"workload": "64^3 cells, 2-point rule (2097152 sources), g at all 262144 cell centres"}
    outs = {}
    # leaf 512 points (4^3 cells) is the faster split; leaf 64 (2^3 cells)
    # moves the work into the M2L (121 GFLOP at p = 10)
    for tag, prec, p, leaf in (("mixed", G.GRAV_MIXED, 10, 512), ("fp64", G.GRAV_FP64, 12, 512),
                               ("mixed_leaf64", G.GRAV_MIXED, 10, 64)):
        plan = G.Plan(G.PlanSpec(n=(n, n, n), h=grid.h, quad_order=2, voxel_centres=True, components=3, p=p,
                                 leaf_size=leaf, precision=prec))
        out = torch.empty(plan.out_shape, dtype=torch.float64, device="cuda")
        ms, lat = timed_steps(plan, rho, out, args.steps, args.warmup)
        stg = stage_profile(plan, rho, out, 5)
        outs[tag] = gather_rows(out, idx)
        row[tag] = {"p": p, "leaf_points": leaf, "value": M / (ms * 1e-3), "ms_per_step": ms,
                    "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "stages_ms": stg,
                    "roofline": roofline(plan, stg, p, prec, None)}
        del plan, out
    if not args.no_cpu:
        import oracle
        ref = oracle.forward(rho_h, grid.origin, grid.h, 2, grid.centres()[idx], comps=3)
        for tag in outs:
            row[tag]["rel_err"] = oracle.rel_l2(outs[tag], ref)
    return row


def batched128(args):
    """32 density models (8 blobs each, seeds 2000 + b) on one 128^3-cell
    tree, gz at 256 x 256 stations at z = 1.1: the mixed-precision batched
    solve (p = 10) against the FP64 FMM (p = 14), batched and as 32 plain
    single-model solves; the adjoint of each (the inversion gradient)."""
    import numpy as np
    import torch

    import paper_1107_5951_amd as G
    import workloads as W
    n, B = 128, 32
    grid = W.Grid.unit(n)
    st = W.stations(256, 1.1)
    rhos = np.stack([W.gaussian_blobs(grid, 8, 2000 + b) for b in range(B)])
    r = torch.as_tensor(rhos, device="cuda")
    sidx = W.sample_indices(st.shape[0], args.sample, seed=7)
    row = {"workload": "128^3 cells, 1-point rule, B=32 models on one tree, gz at 256x256 stations"}
    samples = {}
    for tag, prec, p in (("mixed", G.GRAV_MIXED, 10), ("fp64", G.GRAV_FP64, 14)):
        plan = G.Plan(G.PlanSpec(n=(n, n, n), h=grid.h, points=st, components=1, p=p, leaf_size=64, batch=B,
                                 precision=prec))
        out = torch.empty(plan.out_shape, dtype=torch.float64, device="cuda")
        ms, lat = timed_steps(plan, r, out, 10, 2)
        stg = stage_profile(plan, r, out, 3)
        samples[tag] = out[:4].index_select(1, torch.as_tensor(sidx, device="cuda"))[..., 0].cpu().numpy()
        row[tag] = {"p": p, "value": B * st.shape[0] / (ms * 1e-3), "ms_per_step": ms,
                    "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "stages_ms": stg,
                    "roofline": roofline(plan, stg, p, prec, None)}
        adj_ms, adj_st = adjoint_profile(plan, plan.out_shape, 5)
        row[tag]["adjoint_ms"] = adj_ms
        row[tag]["adjoint_stages_ms"] = adj_st
        # one inversion iteration: forward, misfit, adjoint (the gradient)
        row[tag]["inversion_step_ms"] = ms + adj_ms
        del plan, out
        torch.cuda.empty_cache()
    # the plain FP64 FMM: one model per solve, 32 solves
    plan1 = G.Plan(G.PlanSpec(n=(n, n, n), h=grid.h, points=st, components=1, p=14, leaf_size=64,
                              precision=G.GRAV_FP64))
    out1 = torch.empty(plan1.out_shape, dtype=torch.float64, device="cuda")
    for b in range(2):
        plan1.eval(r[b], out1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for b in range(B):
        plan1.eval(r[b], out1)
    e1.record()
    torch.cuda.synchronize()
    ms1 = e0.elapsed_time(e1)
    row["fp64_single_x32"] = {"p": 14, "ms_for_32": ms1, "value": B * st.shape[0] / (ms1 * 1e-3)}
    row["mixed_batched_speedup_vs_fp64_single"] = ms1 / row["mixed"]["ms_per_step"]
    del plan1, out1
    if not args.no_cpu:
        import oracle
        ref = oracle.forward(rhos[:4], grid.origin, grid.h, 1, st[sidx], comps=1)[..., 0]
        for tag in ("mixed", "fp64"):
            row[tag]["rel_err"] = oracle.rel_l2(samples[tag], ref)
            row[tag]["rel_err_models_x_stations"] = "4 x %d" % len(sidx)
    return row


# ----------------------------------------------------------------------------
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


def scattered(args):
    """Explicit sources: 2,097,152 scattered points (seed 1006, denser towards
    z = 0) with volumes of a rough partition of the unit cube, a density per
    point, gz at 256 x 256 stations at z = 1.1 and at 65,536 scattered points
    inside; the octree framed by a 128^3 mesh (leaves of 4^3 cells, about 64
    sources).  Mixed p = 10 and FP64 p = 14, forward and adjoint."""
    import numpy as np
    import torch

    import paper_1107_5951_amd as G
    import workloads as W
    rng = np.random.default_rng(1006)
    N = 1 << 21
    src = rng.uniform(0.0, 1.0, size=(N, 3)) ** np.array([1.0, 1.0, 1.5])
    vol = rng.uniform(0.5, 1.5, size=N) / N
    dens = np.sin(3 * src[:, 0]) + np.cos(2 * src[:, 1]) * src[:, 2]
    tg = np.concatenate([W.stations(256, 1.1), rng.uniform(0.0, 1.0, size=(65536, 3))])
    sidx = W.sample_indices(tg.shape[0], 1024, seed=7)
    row = {"workload": "2097152 scattered sources with volumes (128^3 frame, leaf 4^3 cells), gz at 256^2 "
                       "stations + 65536 interior points"}
    r = torch.as_tensor(dens[None], device="cuda")
    samples = {}
    for tag, prec, p in (("mixed", G.GRAV_MIXED, 10), ("fp64", G.GRAV_FP64, 14)):
        t0 = time.perf_counter()
        plan = G.Plan(G.PlanSpec(n=(128, 128, 128), h=1 / 128, points=tg, components=1, p=p, leaf_size=64,
                                 precision=prec, sources=src, source_volumes=vol))
        plan_s = time.perf_counter() - t0
        out = torch.empty(plan.out_shape, dtype=torch.float64, device="cuda")
        ms, lat = timed_steps(plan, r, out, 10, 2)
        stg = stage_profile(plan, r, out, 3)
        samples[tag] = out[0, torch.as_tensor(sidx, device="cuda"), 0].cpu().numpy()
        adj_ms, adj_st = adjoint_profile(plan, plan.out_shape, 3)
        m2l_pairs, p2p_pairs, _ = plan.work()
        row[tag] = {"p": p, "value": tg.shape[0] / (ms * 1e-3), "ms_per_step": ms, "p50_ms": pct(lat, 50),
                    "p99_ms": pct(lat, 99), "plan_s": plan_s, "stages_ms": stg, "adjoint_ms": adj_ms,
                    "adjoint_stages_ms": adj_st, "p2p_point_pairs": p2p_pairs, "m2l_box_pairs": m2l_pairs}
        del plan, out
        torch.cuda.empty_cache()
    if not args.no_cpu:
        import oracle
        ref = oracle.points(src, dens * vol, tg[sidx], comps=4)[:, 3]
        for tag in samples:
            row[tag]["rel_err"] = oracle.rel_l2(samples[tag], ref)
        row["rel_err_targets"] = len(sidx)
    return row


def serving(args):
    """The serving workload: a seeded Poisson trace (rate 50/s, seed 1005) of
    forward and adjoint requests (50/50) on meshes n = round(exp U[ln 32,
    ln 192]), q in {1, 2}, gz at n x n stations, mixed precision p = 10;
    graph-captured solves with continuous batching, served back to back
    (capacity) and at the trace's arrival times (latency under load)."""
    from paper_1107_5951_amd import serve
    print(json.dumps(serve.benchmark(args.serve, log=say)), flush=True)


def crossover(args):
    """Summation vs FMM as the number of stations grows (cf. the paper's
    crossover discussion, Sec. 4): a fixed 64^3 mesh, 1-point rule, gz at
    ns x ns stations at z = 1.1, mixed precision p = 10; the summation by the
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
        plan = G.Plan(G.PlanSpec(n=(n, n, n), h=grid.h, points=W.stations(ns, 1.1), components=1, p=10,
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
    if args.crossover:
        crossover(args)
        return
    if args.serve:
        serving(args)
        return
    if args.paper_sequence:
        paper_sequence(args)
        return
    if args.batched_only:
        say("batched 128^3 workload")
        print(json.dumps({"batched128_b32": batched128(args)}), flush=True)
        return

    res = headline(args)
    if not args.no_extra and not args.timed_only:
        say("64^3 volume workload")
        res["volume64_q2"] = volume64(args)
        torch.cuda.empty_cache()
        say("batched 128^3 workload")
        res["batched128_b32"] = batched128(args)
        torch.cuda.empty_cache()
        say("scattered sources")
        res["scattered_sources"] = scattered(args)
    line = json.dumps(res)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
