"""Replanning server: continuous batching over resident roadmaps.

Requests arrive over time; each names a sample set (dim, n, sample seed) and
a query (start, goal, boxes, lambda).  Roadmaps stay resident on the device
in an LRU cache under a byte budget (a roadmap with requests in flight is
never evicted); the native engine (``gmt_engine_*``) admits queries by the
device memory of their workspaces, forms batches from whatever is queued
when a stream frees up, and overlaps batches on the device.  Latency is
arrival to completion; throughput is completed queries over the makespan.
"""

from __future__ import annotations

import collections
import gc
import json
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, Hashable, List, Optional

import numpy as np

from . import gmt


def roadmap_bytes(n: int, dim: int, kind: int, nnz: int, cap: int = 0) -> int:
    """Device bytes of a roadmap, estimated before it is built: samples, row
    pointers and records.  Euclidean: row lengths and `cap` 8-byte slots per
    row (the expected degree, or nnz / n when cap is not given) plus 256
    padding slots.  Otherwise: columns, 12-byte (cost, column) records plus
    256 padding records, and for the double integrator arrival times, the
    transposed table and 8-float states.  A built roadmap reports its own
    figure (Roadmap.device_bytes)."""
    b = 4 * dim * n + 4 * (n + 1)
    if kind == gmt.GMT_COST_EUCLIDEAN:
        slots = n * cap if cap else nnz
        return b + 4 * n + 8 * (slots + 256)
    b += 4 * nnz + 12 * (nnz + 256)
    if kind == gmt.GMT_COST_DOUBLE_INTEGRATOR:
        b += 8 * nnz + 4 * (n + 1) + 4 * nnz + 32 * n  # arrival times, transposed table, 8-float states
    return b


class RoadmapCache:
    """LRU of resident roadmaps under ``budget`` bytes, with pin counts."""

    def __init__(self, budget: int, build: Callable[[Hashable], "gmt.Roadmap"],
                 size_of: Callable[["gmt.Roadmap"], int] = None):
        self.budget = int(budget)
        self.build = build
        self.size_of = size_of or (lambda rm: rm.device_bytes)
        self.items: "collections.OrderedDict[Hashable, list]" = collections.OrderedDict()
        self.bytes = 0
        self.hits = 0
        self.misses = 0
        self.evictions = 0
        self.lock = threading.Lock()

    def acquire(self, key: Hashable):
        """Roadmap for ``key``, pinned until ``release(key)``."""
        with self.lock:
            it = self.items.get(key)
            if it is not None:
                self.items.move_to_end(key)
                it[2] += 1
                self.hits += 1
                return it[0]
            self.misses += 1
        rm = self.build(key)
        size = self.size_of(rm)
        with self.lock:
            self._evict(size)
            self.items[key] = [rm, size, 1]
            self.bytes += size
        return rm

    def release(self, key: Hashable) -> None:
        with self.lock:
            self.items[key][2] -= 1

    def _evict(self, need: int) -> None:
        for k in list(self.items.keys()):
            if self.bytes + need <= self.budget:
                return
            rm, size, pins = self.items[k]
            if pins > 0:
                continue
            del self.items[k]
            self.bytes -= size
            self.evictions += 1
            if hasattr(rm, "free"):
                rm.free()

    def clear(self) -> None:
        with self.lock:
            for rm, _, _ in self.items.values():
                if hasattr(rm, "free"):
                    rm.free()
            self.items.clear()
            self.bytes = 0


@dataclass
class Request:
    arrival_s: float
    key: Hashable                      # roadmap key
    make_query: Callable[["gmt.Roadmap"], "gmt.BatchQuery"]
    tag: object = None


@dataclass
class Served:
    tag: object
    status: int
    path: np.ndarray
    path_cost: float
    latency_ms: float
    queue_wait_ms: float


@dataclass
class ServeReport:
    served: List[Served]
    makespan_s: float
    plans_per_s: float
    p50_ms: float
    p99_ms: float
    engine: dict = field(default_factory=dict)
    cache: dict = field(default_factory=dict)


class ReplanServer:
    def __init__(self, build_roadmap: Callable[[Hashable], "gmt.Roadmap"], opts: "gmt.gmt_plan_opts",
                 engine_budget: int, roadmap_budget: int, slots: int = 4, max_batch: int = 256,
                 workgroups: int = 0, path_cap: int = 512):
        self.cache = RoadmapCache(roadmap_budget, build_roadmap)
        self.engine = gmt.Engine(engine_budget, opts, slots=slots, max_batch=max_batch,
                                 workgroups=workgroups)
        self.path_cap = path_cap

    def serve(self, requests: List[Request], realtime: bool = True, record: Optional[str] = None) -> ServeReport:
        """Replay ``requests`` at their arrival times (``realtime``) or all at
        once, and collect every result.  ``record``: a file to which one JSON
        line per request is appended as it completes (tag, roadmap key,
        arrival, submit and completion times on the engine's steady clock,
        latency, status, iterations, path length and cost)."""
        # the interpreter's cyclic collector stays off while requests are
        # replayed: a full collection over a large heap stalls the submitter
        # thread for tens of milliseconds, which would hold back arrivals
        gc_was_on = gc.isenabled()
        gc.disable()
        try:
            return self._serve(requests, realtime, record)
        finally:
            if gc_was_on:
                gc.enable()

    def _serve(self, requests: List[Request], realtime: bool, record: Optional[str]) -> ServeReport:
        out = open(record, "a") if record else None
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        t0 = gmt.gmt_steady_ns() + 2_000_000  # start 2 ms from now
        tickets: Dict[int, tuple] = {}
        lock = threading.Lock()

        errors: List[BaseException] = []

        def submitter():
            try:
                submit_all()
            except BaseException as e:  # surfaced by the collector
                errors.append(e)

        def submit_all():
            for r in reqs:
                at = t0 + int(r.arrival_s * 1e9) if realtime else t0
                while True:
                    now = gmt.gmt_steady_ns()
                    if now >= at:
                        break
                    if at - now > 200_000:
                        time.sleep((at - now - 100_000) / 1e9)
                rm = self.cache.acquire(r.key)
                tk = self.engine.submit(r.make_query(rm), self.path_cap)
                with lock:
                    tickets[tk] = (r, at)

        th = threading.Thread(target=submitter, daemon=True)
        th.start()
        served: List[Served] = []
        last_done = t0
        while len(served) < len(reqs):
            got = self.engine.poll_any(2000, self.path_cap)  # completion order; releases the GIL while waiting
            if got is None:
                if errors and not th.is_alive():
                    raise errors[0]
                continue
            tk, res = got
            while True:  # the submitter records a ticket just after submit returns it
                with lock:
                    entry = tickets.pop(tk, None)
                if entry is not None:
                    break
                time.sleep(0)
            r, at = entry
            self.cache.release(r.key)
            done = res.work["done_ns"]
            last_done = max(last_done, done)
            served.append(Served(r.tag, res.status, res.path, res.path_cost, (done - at) / 1e6,
                                 (res.work["submit_ns"] - at) / 1e6))
            if out:
                out.write(json.dumps({"tag": str(r.tag), "key": str(r.key), "arrival_ns": at,
                                      "submit_ns": res.work["submit_ns"], "done_ns": done,
                                      "latency_ms": round((done - at) / 1e6, 4), "status": int(res.status),
                                      "iterations": int(res.iters), "path_len": len(res.path),
                                      "path_cost": float(res.path_cost)}) + "\n")
        th.join()
        if out:
            out.close()
        lat = np.array([s.latency_ms for s in served]) if served else np.zeros(1)
        first = t0
        span = max(last_done - first, 1) / 1e9
        return ServeReport(served, span, len(served) / span, float(np.percentile(lat, 50)),
                           float(np.percentile(lat, 99)), self.engine.stats(),
                           {"hits": self.cache.hits, "misses": self.cache.misses,
                            "evictions": self.cache.evictions, "bytes": self.cache.bytes})

    def close(self) -> None:
        self.engine.close()
        self.cache.clear()
