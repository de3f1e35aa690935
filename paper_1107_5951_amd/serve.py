"""Serving loop for gravity inversion workloads on one GPU.

Requests are independent forward or adjoint solves: a density on an
n x n x n unit-cube mesh (1- or 2-point rule) mapped to gz at n x n stations
at z = 1.1 (forward), or gz residuals at those stations mapped back to a
density gradient (adjoint, the transpose of the forward map).

* Plans stay resident: a slot is one plan (mesh size, rule, batch size) with
  its own HIP stream, static input and output buffers and, by default, one
  captured HIP graph per direction, so serving a request is a device copy of
  its input, a graph replay and a device copy of its output.
* Admission by HBM footprint: a slot's bytes are the plan's reported
  footprint (grav_plan_bytes) plus its static buffers.  A request whose slot
  does not fit the budget waits until enough in-flight work finishes for
  idle slots to be evicted (least recently used first); it is rejected only
  when its slot alone exceeds the budget.
* Continuous batching: whenever a stream slot frees up, the oldest waiting
  request is started together with the other waiting requests of the same
  mesh, rule and direction, as one batched solve (batch sizes 1, 2, 4, 8;
  unused batch members are computed and ignored; a resident slot is used
  before a new batch size is built).  Requests that arrive
  while others run are admitted as slots and memory free up, and their work
  overlaps on the device with the work already in flight.

Results do not depend on what else is in flight: each slot's work uses only
its own plan and buffers, every kernel is deterministic, and a batched solve
computes each model independently (its rounding can differ from a
single-model solve only in the order of the M2L partial sums).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import GRAV_MIXED, Plan, PlanSpec

BATCH_SIZES = (1, 2, 4, 8)


@dataclasses.dataclass
class Request:
    n: int                      # cells per axis of the unit-cube mesh
    q: int                      # 1- or 2-point rule per axis
    data: object                # forward: float64 HIP tensor [n, n, n] (rho);
                                # adjoint: float64 HIP tensor [n * n] (gz residuals)
    kind: str = "forward"       # "forward" or "adjoint"
    arrival: float = 0.0        # seconds, trace time


@dataclasses.dataclass
class Result:
    index: int
    kind: str
    out: object = None          # forward: [n * n] gz; adjoint: [n, n, n] drho
    t_arrive: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    batch: int = 1
    error: Optional[str] = None


def station_grid(ns: int, z: float = 1.1) -> np.ndarray:
    h = 1.0 / ns
    c = (np.arange(ns) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1)


def plan_spec(n: int, q: int, batch: int = 1, p: int = 10, precision: int = GRAV_MIXED,
              leaf_size: int = 64) -> PlanSpec:
    """The plan a request of mesh n and rule q is served with."""
    return PlanSpec(n=(n, n, n), h=1.0 / n, quad_order=q, points=station_grid(n), components=1, p=p,
                    leaf_size=leaf_size * q ** 3, precision=precision, batch=batch)


class Slot:
    """A resident plan with its stream, static buffers and captured graphs."""

    def __init__(self, n: int, q: int, batch: int, p: int, precision: int, graphs: bool):
        import torch
        self.torch = torch
        self.key = (n, q, batch)
        self.plan = Plan(plan_spec(n, q, batch, p, precision))
        self.stream = torch.cuda.Stream()  # default priority
        dev = torch.device("cuda")
        self.rho = torch.zeros(self.plan.rho_shape, dtype=torch.float64, device=dev)
        self.g = torch.zeros(self.plan.out_shape, dtype=torch.float64, device=dev)
        self.resid = torch.zeros(self.plan.out_shape, dtype=torch.float64, device=dev)
        self.drho = torch.zeros(self.plan.rho_shape, dtype=torch.float64, device=dev)
        resident, per_call = self.plan.bytes()
        self.nbytes = resident + per_call + 8 * (2 * self.rho.numel() + 2 * self.g.numel())
        self.graphs: Dict[str, object] = {}
        self.event = None           # completion of the last launch
        self.last_used = 0.0
        self._run("forward")        # eager warm-up on the slot's stream
        self._run("adjoint")
        if graphs:
            self._capture()
        torch.cuda.synchronize()

    def _run(self, kind: str) -> None:
        if kind == "forward":
            self.plan.eval(self.rho, self.g, stream=self.stream)
        else:
            self.plan.adjoint(self.resid, self.drho, stream=self.stream)

    def _capture(self) -> None:
        torch = self.torch
        torch.cuda.synchronize()
        for kind in ("forward", "adjoint"):
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=self.stream):
                self._run(kind)
            self.graphs[kind] = graph

    @property
    def busy(self) -> bool:
        return self.event is not None and not self.event.query()

    def launch(self, kind: str, reqs: List[Request], src_stream) -> List[object]:
        """Copy the requests' inputs into the static buffers, run the solve
        (graph replay or eager) and copy each request's output out, all on the
        slot's stream; returns the output tensors."""
        torch = self.torch
        s = self.stream
        s.wait_stream(src_stream)  # inputs were produced on the caller's stream
        outs = []
        with torch.cuda.stream(s):
            for b, r in enumerate(reqs):
                if kind == "forward":
                    self.rho[b].copy_(r.data.reshape(self.rho.shape[1:]))
                else:
                    self.resid[b].copy_(r.data.reshape(self.resid.shape[1:]))
                r.data.record_stream(s)
            if kind in self.graphs:
                self.graphs[kind].replay()
            else:
                self._run(kind)
            for b in range(len(reqs)):
                src = self.g[b, :, 0] if kind == "forward" else self.drho[b]
                outs.append(src.clone())
            self.event = torch.cuda.Event()
            self.event.record(s)
        return outs

    def close(self) -> None:
        if self.event is not None:
            self.event.synchronize()
        self.graphs.clear()
        self.plan.close()


class GravServer:
    """Continuous-batching server for forward and adjoint requests."""

    def __init__(self, budget_bytes: int = 64 << 30, max_inflight: int = 4, p: int = 10,
                 precision: int = GRAV_MIXED, batching: bool = True, graphs: bool = True):
        import torch
        self.torch = torch
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.p, self.precision = p, precision
        self.batching, self.use_graphs = batching, graphs
        self.slots: "collections.OrderedDict[Tuple[int, int, int], Slot]" = collections.OrderedDict()
        self._footprint: Dict[Tuple[int, int, int], int] = {}
        self.stats = collections.Counter()

    # ------------------------------------------------------------ admission
    @property
    def used(self) -> int:
        return sum(s.nbytes for s in self.slots.values())

    def _slot(self, n: int, q: int, batch: int) -> Optional[Slot]:
        """The resident slot for (n, q, batch), built if the budget allows
        (evicting idle slots, least recently used first); None if it has to
        wait for in-flight work to finish; MemoryError if it can never fit."""
        key = (n, q, batch)
        if key in self.slots:
            self.slots.move_to_end(key)
            self.stats["slot_hits"] += 1
            return self.slots[key]
        need = self._footprint.get(key)
        if need is not None:
            if need > self.budget:
                raise MemoryError("a plan for n=%d q=%d batch %d needs %d bytes, budget %d"
                                  % (n, q, batch, need, self.budget))
            if not self._make_room(need):
                self.stats["admission_waits"] += 1
                return None
        slot = Slot(n, q, batch, self.p, self.precision, self.use_graphs)
        self._footprint[key] = slot.nbytes
        self.stats["slot_builds"] += 1
        if slot.nbytes > self.budget:
            slot.close()
            raise MemoryError("a plan for n=%d q=%d batch %d needs %d bytes, budget %d"
                              % (n, q, batch, slot.nbytes, self.budget))
        if not self._make_room(slot.nbytes):
            slot.close()
            self.stats["admission_waits"] += 1
            return None
        self.slots[key] = slot
        return slot

    def _batch_size(self, n: int, q: int, waiting: int) -> int:
        """Batch size for `waiting` same-plan requests: the smallest resident
        slot that takes them all; else a resident slot that takes at least
        half of them (the rest go in the next round); else the smallest batch
        size that fits them all (a new slot: a plan and two graph captures,
        worth it only when it replaces several launches)."""
        k = min(waiting, BATCH_SIZES[-1])
        have = [b for b in BATCH_SIZES if (n, q, b) in self.slots]
        up = [b for b in have if b >= k]
        if up:
            return min(up)
        if have and 2 * max(have) >= k:
            return max(have)
        return next(b for b in BATCH_SIZES if b >= k)

    def _make_room(self, need: int) -> bool:
        """Evict idle slots (least recently used first) until `need` more bytes
        fit the budget; False if only in-flight slots are left to evict."""
        while self.used + need > self.budget:
            idle = [k for k, s in self.slots.items() if not s.busy]
            if not idle:
                return False
            self.slots.pop(idle[0]).close()
            self.stats["evictions"] += 1
        return True

    # ------------------------------------------------------------ serving
    def run(self, requests: List[Request], realtime: bool = False) -> Tuple[List[Result], dict]:
        """Serve a trace.  realtime=True admits each request at its arrival
        time (latency under load); otherwise all requests are waiting from the
        start (capacity).  Returns the results in request order and summary
        statistics (latency from arrival to completion)."""
        torch = self.torch
        src = torch.cuda.current_stream()
        results = [Result(i, r.kind) for i, r in enumerate(requests)]
        waiting: "collections.deque[int]" = collections.deque()
        inflight: List[Tuple[Slot, List[int]]] = []
        nxt = 0
        t0 = time.perf_counter()
        self.stats.clear()

        def now():
            return time.perf_counter() - t0

        def reap():
            nonlocal inflight
            keep = []
            for slot, idx in inflight:
                if slot.event.query():
                    t = now()
                    for i in idx:
                        results[i].t_done = t
                else:
                    keep.append((slot, idx))
            inflight = keep

        while nxt < len(requests) or waiting or inflight:
            # admit arrivals
            while nxt < len(requests) and (not realtime or requests[nxt].arrival <= now()):
                results[nxt].t_arrive = requests[nxt].arrival if realtime else 0.0
                waiting.append(nxt)
                nxt += 1
            reap()
            started = False
            tried = set()
            # the oldest waiting request of each (mesh, rule, direction) in
            # arrival order, with the waiting requests that share its plan
            for i in list(waiting):
                if len(inflight) >= self.max_inflight:
                    break
                head = requests[i]
                kind, key = head.kind, (head.n, head.q)
                if (kind, key) in tried or i not in waiting:
                    continue
                tried.add((kind, key))
                group = [j for j in waiting if requests[j].kind == kind and
                         (requests[j].n, requests[j].q) == key] if self.batching else [i]
                batch = self._batch_size(head.n, head.q, len(group))
                group = group[:batch]
                try:
                    slot = self._slot(head.n, head.q, batch)
                except MemoryError as e:
                    for j in group:
                        results[j].error = str(e)
                        results[j].t_done = now()
                        waiting.remove(j)
                    continue
                if slot is None or slot.busy:
                    continue  # memory or this plan's stream frees up later
                t = now()
                outs = slot.launch(kind, [requests[j] for j in group], src)
                for j, o in zip(group, outs):
                    results[j].out = o
                    results[j].t_start = t
                    results[j].batch = batch
                    waiting.remove(j)
                inflight.append((slot, group))
                slot.last_used = t
                self.stats["batches"] += 1
                self.stats["batched_requests"] += len(group)
                started = True
            if not started:
                if inflight and (waiting or nxt >= len(requests)):
                    inflight[0][0].event.synchronize()
                elif realtime and nxt < len(requests):
                    time.sleep(min(2e-4, max(0.0, requests[nxt].arrival - now())))
        torch.cuda.synchronize()
        wall = now()
        ok = [r for r in results if r.error is None]
        lat = sorted((r.t_done - r.t_arrive) * 1e3 for r in ok)
        pick = lambda q: lat[min(len(lat) - 1, int(round(q / 100.0 * (len(lat) - 1))))] if lat else 0.0
        evals = sum(requests[r.index].n ** 2 for r in ok)
        stats = {"requests": len(results), "served": len(ok), "rejected": len(results) - len(ok),
                 "forward": sum(1 for r in ok if r.kind == "forward"),
                 "adjoint": sum(1 for r in ok if r.kind == "adjoint"),
                 "wall_s": wall, "requests_per_s": len(ok) / wall, "gz_evals_per_s": evals / wall,
                 "p50_ms": pick(50), "p99_ms": pick(99), "resident_slots": len(self.slots),
                 "resident_bytes": self.used, "graphs": self.use_graphs}
        stats.update({k: int(v) for k, v in self.stats.items()})
        return results, stats

    def close(self) -> None:
        self.torch.cuda.synchronize()
        for s in self.slots.values():
            s.close()
        self.slots.clear()


def poisson_trace(count: int, rate: float, seed: int, n_min: int = 32, n_max: int = 192,
                  adjoint_fraction: float = 0.5, device: str = "cuda", host_blobs: bool = True) -> List[Request]:
    """Synthetic request trace: Poisson arrivals at `rate` per second, n
    log-uniform on [n_min, n_max], q uniform in {1, 2}, adjoint with
    probability `adjoint_fraction`.  Forward inputs: 8 seeded Gaussian blobs
    (seed + request index) built on the host, or, with host_blobs=False,
    seeded uniform noise drawn on the device (timing runs with large meshes);
    adjoint inputs: seeded standard normal residuals at the n x n stations."""
    import torch

    from workloads import Grid, gaussian_blobs

    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    ns = np.rint(np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=count))).astype(int)
    qs = rng.integers(1, 3, size=count)
    adj = rng.uniform(size=count) < adjoint_fraction
    reqs = []
    for i in range(count):
        n = int(ns[i])
        gen = torch.Generator(device=device).manual_seed(seed + 1 + i)
        if adj[i]:
            data = torch.randn((n * n,), dtype=torch.float64, device=device, generator=gen)
        elif host_blobs:
            data = torch.as_tensor(gaussian_blobs(Grid.unit(n), 8, seed + 1 + i), device=device)
        else:
            data = torch.rand((n, n, n), dtype=torch.float64, device=device, generator=gen)
        reqs.append(Request(n=n, q=int(qs[i]), data=data, kind="adjoint" if adj[i] else "forward",
                            arrival=float(t[i])))
    return reqs


def benchmark(count: int = 3000, rate: float = 50.0, seed: int = 1005, log=None) -> dict:
    """The serving workload: a Poisson trace of forward and adjoint requests
    (50/50), meshes 32^3 .. 192^3, q in {1, 2}, mixed precision at p = 10;
    plans and graphs are built first (timed separately), then the trace is
    served at its arrival times (latency under load, every plan resident),
    then back to back twice (capacity: the second pass, with the batched
    slots the first one built resident)."""
    import torch
    say = log or (lambda msg: None)
    reqs = poisson_trace(count, rate, seed, host_blobs=False)
    srv = GravServer(budget_bytes=128 << 30)
    t0 = time.perf_counter()
    keys = sorted(set((r.n, r.q) for r in reqs))
    for i, key in enumerate(keys):
        srv._slot(key[0], key[1], 1)
        if (i + 1) % 25 == 0 or i + 1 == len(keys):
            say("serving: %d of %d plans and graphs built" % (i + 1, len(keys)))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    _, live = srv.run(reqs, realtime=True)  # at the arrival times, plans resident
    say("serving: pass at arrival times done")
    _, cold = srv.run(reqs)             # back to back; builds the batched slots it needs
    say("serving: first back-to-back pass done (%.1f s)" % cold["wall_s"])
    _, cap = srv.run(reqs)              # back to back again, batched slots resident
    say("serving: second back-to-back pass done (%.1f s)" % cap["wall_s"])
    srv.close()
    cap["first_pass_wall_s"] = cold["wall_s"]
    cap["first_pass_slot_builds"] = cold.get("slot_builds", 0)
    return {"workload": "serving: %d Poisson requests at %g/s (seed %d), forward and adjoint 50/50, n in [32, 192], "
                        "q in {1, 2}, gz at n^2 stations, mixed precision p=10, graph replays, continuous batching"
                        % (count, rate, seed),
            "plans": len(set((r.n, r.q) for r in reqs)), "plan_and_graph_build_s": build_s,
            "capacity": cap, "realtime": live}
