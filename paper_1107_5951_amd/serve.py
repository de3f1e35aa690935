"""Serving loop for many small forward solves on one GPU.

Requests are independent gravity forward models: a density on an n x n x n
unit-cube mesh (1- or 2-point rule) and gz at n x n stations at z = 1.1.
The server keeps a cache of plans keyed by the request's geometry, admits
plans against an HBM budget using their reported footprint
(``grav_plan_bytes``), and keeps several requests in flight on a small pool
of HIP streams.  A plan's workspace serves one call at a time, so every plan
is bound to one stream and its requests run there in arrival order; requests
of different plans overlap.  Results do not depend on what else is in
flight: each evaluation uses only its own plan and buffers, and every kernel
is deterministic.

The transposed (adjoint) solve is not served: ``grav_adjoint`` is switched
off in the library build.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import GRAV_MIXED, Plan, PlanSpec


@dataclasses.dataclass
class Request:
    n: int                      # cells per axis of the unit-cube mesh
    q: int                      # 1- or 2-point rule per axis
    rho: object                 # float64 HIP tensor [n, n, n]
    kind: str = "forward"
    arrival: float = 0.0        # seconds, trace time


@dataclasses.dataclass
class Result:
    index: int
    out: object                 # float64 HIP tensor [n*n, 1] (gz at the stations)
    t_submit: float
    t_done: float = 0.0
    event: object = None


def station_grid(ns: int, z: float = 1.1) -> np.ndarray:
    h = 1.0 / ns
    c = (np.arange(ns) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1)


class PlanCache:
    """LRU cache of plans with an HBM budget on their resident + workspace bytes."""

    def __init__(self, budget_bytes: int, p: int = 10, precision: int = GRAV_MIXED, leaf_size: int = 64):
        self.budget = int(budget_bytes)
        self.p, self.precision, self.leaf_size = p, precision, leaf_size
        self._plans: "collections.OrderedDict[Tuple[int, int], Plan]" = collections.OrderedDict()
        self._bytes: Dict[Tuple[int, int], int] = {}
        self.hits = self.misses = self.evictions = 0

    @property
    def used(self) -> int:
        return sum(self._bytes.values())

    def get(self, n: int, q: int) -> Plan:
        key = (n, q)
        if key in self._plans:
            self._plans.move_to_end(key)
            self.hits += 1
            return self._plans[key]
        self.misses += 1
        spec = PlanSpec(n=(n, n, n), h=1.0 / n, quad_order=q, points=station_grid(n), components=1,
                        p=self.p, leaf_size=self.leaf_size * q ** 3, precision=self.precision)
        plan = Plan(spec)
        resident, per_call = plan.bytes()
        need = resident + per_call
        if need > self.budget:
            plan.close()
            raise MemoryError("plan for n=%d q=%d needs %d bytes, budget %d" % (n, q, need, self.budget))
        while self._plans and self.used + need > self.budget:
            old, victim = self._plans.popitem(last=False)
            del self._bytes[old]
            victim.close()
            self.evictions += 1
        self._plans[key] = plan
        self._bytes[key] = need
        return plan

    def close(self) -> None:
        for plan in self._plans.values():
            plan.close()
        self._plans.clear()
        self._bytes.clear()


class GravServer:
    """Dispatch forward requests to a pool of streams, one stream per plan."""

    def __init__(self, n_streams: int = 4, budget_bytes: int = 64 << 30, p: int = 10,
                 precision: int = GRAV_MIXED):
        import torch
        self.torch = torch
        self.cache = PlanCache(budget_bytes, p=p, precision=precision)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]  # default priority
        self._stream_of: Dict[Tuple[int, int], int] = {}
        self._next = 0

    def _stream_for(self, key: Tuple[int, int]):
        if key not in self._stream_of:
            self._stream_of[key] = self._next % len(self.streams)
            self._next += 1
        return self.streams[self._stream_of[key]]

    def submit(self, index: int, req: Request) -> Result:
        torch = self.torch
        if req.kind != "forward":
            raise NotImplementedError("only forward requests are served")
        plan = self.cache.get(req.n, req.q)
        s = self._stream_for((req.n, req.q))
        t0 = time.perf_counter()
        # the request's input was produced on the current stream
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            out = torch.empty(plan.out_shape, dtype=torch.float64, device="cuda")
            plan.eval(req.rho, out, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        req.rho.record_stream(s)
        return Result(index, out[0], t0, event=ev)

    def run(self, requests: List[Request], realtime: bool = False) -> Tuple[List[Result], dict]:
        """Serve a trace.  realtime=True waits for each arrival time (latency
        under load); otherwise requests are submitted back to back
        (capacity).  Returns the results and summary statistics."""
        results: List[Result] = []
        pending: List[Result] = []
        t_start = time.perf_counter()

        def reap(block: bool):
            nonlocal pending
            keep = []
            for r in pending:
                if block:
                    r.event.synchronize()
                if r.event.query():
                    r.t_done = time.perf_counter()
                else:
                    keep.append(r)
            pending = keep

        for i, req in enumerate(requests):
            if realtime:
                while time.perf_counter() - t_start < req.arrival:
                    reap(False)
                    time.sleep(0.0002)
            r = self.submit(i, req)
            if realtime:
                r.t_submit = t_start + req.arrival
            results.append(r)
            pending.append(r)
            reap(False)
        reap(True)
        wall = time.perf_counter() - t_start
        lat = sorted((r.t_done - r.t_submit) * 1e3 for r in results)
        pick = lambda q: lat[min(len(lat) - 1, int(round(q / 100.0 * (len(lat) - 1))))] if lat else 0.0
        evals = sum(r.out.shape[0] for r in results)
        stats = {"requests": len(results), "wall_s": wall, "requests_per_s": len(results) / wall,
                 "gz_evals_per_s": evals / wall, "p50_ms": pick(50), "p99_ms": pick(99),
                 "plan_hits": self.cache.hits, "plan_misses": self.cache.misses,
                 "plan_evictions": self.cache.evictions, "plan_bytes": self.cache.used}
        return results, stats

    def close(self) -> None:
        self.torch.cuda.synchronize()
        self.cache.close()


def poisson_trace(count: int, rate: float, seed: int, n_min: int = 32, n_max: int = 192,
                  device: str = "cuda", host_blobs: bool = True) -> List[Request]:
    """Synthetic request trace: Poisson arrivals, n log-uniform on
    [n_min, n_max], q uniform in {1, 2}.  Densities: 8 seeded Gaussian blobs
    (seed + request index) built on the host, or, with host_blobs=False,
    seeded uniform noise drawn on the device (for timing runs with large
    meshes, where host generation would dominate)."""
    import torch

    from workloads import Grid, gaussian_blobs

    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    ns = np.rint(np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=count))).astype(int)
    qs = rng.integers(1, 3, size=count)
    reqs = []
    for i in range(count):
        n = int(ns[i])
        if host_blobs:
            rho = torch.as_tensor(gaussian_blobs(Grid.unit(n), 8, seed + 1 + i), device=device)
        else:
            gen = torch.Generator(device=device).manual_seed(seed + 1 + i)
            rho = torch.rand((n, n, n), dtype=torch.float64, device=device, generator=gen)
        reqs.append(Request(n=n, q=int(qs[i]), rho=rho, arrival=float(t[i])))
    return reqs
