"""Serving loop: resident graphs, admission by memory, continuous batching.

Queries (graph, source) arrive over time.  The scheduler admits them as
execution slots and device memory allow: workspaces are pooled per graph and
charged against a byte budget while they exist, and every in-flight run also
charges its output array until it completes; idle workspaces of other graphs
are evicted when a query needs room.  Queued queries for the same
low-diameter graph are merged into one batched multi-source run (up to 256
sources, uint8 levels, and no more than fit in a set share of the budget)
when that is cheaper than running them one by one: the scheduler keeps the
device time of single and batched runs per graph, and a batch of k needs
k x (single time) >= (batch time), since a batch's passes over the graph cost
nearly the same for 4 sources as for 256.  Other queries run single-source on
their own stream.
Queries that arrive while others are on the GPU are admitted as soon as a
slot and memory free up, so their work overlaps on the device.

Every answer is the level array of its query (int32, -1 unreached), the
same whether it ran alone, in a batch or next to other queries.  A query
whose launch or collection fails is answered with an error (``Query.error``,
no result); its workspace is dropped and the loop keeps serving the others.

The scheduler talks to an executor (``GpuExecutor`` runs the HIP library;
tests substitute a CPU executor) and to a clock, so its admission and
batching logic is testable without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable

import numpy as np


@dataclasses.dataclass
class Query:
    qid: int
    graph: str
    source: int
    arrival: float                  # seconds on the scheduler's clock
    admitted: float | None = None
    finished: float | None = None
    batched: bool = False
    result: object = None           # int32 levels (executor-specific array type)
    error: str | None = None        # why the query failed (result is then None)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class GraphInfo:
    name: str
    n: int
    m: int
    batchable: bool                 # low diameter: levels fit in a byte for every source
    ws_bytes_single: int
    ws_bytes_batch: int


class Scheduler:
    """Continuous-batching request loop over an executor."""

    def __init__(self, executor, budget_bytes: int, max_inflight: int = 4, batch_max: int = 256,
                 batch_min: int = 2, clock: Callable[[], float] = time.perf_counter, batch_share: float = 0.5,
                 keep_results: bool = True):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.batch_max = batch_max
        self.batch_min = batch_min
        self.batch_share = batch_share      # a batch (workspace + output) takes at most this part of the budget
        self.keep_results = keep_results    # False: answers are dropped once delivered (long runs)
        self.clock = clock
        self.used = 0
        self.pool: dict[tuple[str, int], list] = collections.defaultdict(list)  # idle workspaces
        self.pool_bytes: dict[int, int] = {}
        self.inflight: list = []
        self.pending: collections.deque[Query] = collections.deque()
        self.done: list[Query] = []
        self.stats = collections.Counter()
        self.cost: dict[tuple[str, bool], float] = {}  # device seconds per run, (graph, batched)

    # ---- memory ---------------------------------------------------------------------------
    @staticmethod
    def _ws_cost(info: GraphInfo, kind: int) -> int:
        return info.ws_bytes_batch if kind > 1 else info.ws_bytes_single

    @staticmethod
    def _out_cost(info: GraphInfo, k: int) -> int:
        return info.n * k if k > 1 else 4 * info.n     # uint8 [n][k], or int32 levels

    def _batch_cap(self, info: GraphInfo) -> int:
        """Most sources one batch on this graph may take within its share of the budget."""
        room = int(self.budget * self.batch_share) - info.ws_bytes_batch
        return max(0, min(self.batch_max, room // max(info.n, 1)))

    def _acquire(self, name: str, k: int):
        """An idle workspace for (graph, k-class), or a new one, plus the run's output, if the
        budget allows; None otherwise.  A single-source run may evict idle workspaces of other
        graphs (batched ones first); a batch only uses what is free, so that the large batched
        workspaces never push out the single-source ones every graph keeps needing."""
        info = self.ex.info[name]
        kind = 256 if k > 1 else 1
        pooled = bool(self.pool[(name, kind)])
        need = self._out_cost(info, k) + (0 if pooled else self._ws_cost(info, kind))
        while kind == 1 and self.used + need > self.budget and self._evict_one(exclude=(name, kind)):
            pass
        if self.used + need > self.budget:
            return None
        self.used += need
        if pooled:
            return self.pool[(name, kind)].pop()
        t0 = self.clock()
        ws = self.ex.create(name, kind)
        self.stats["create_ms"] += (self.clock() - t0) * 1e3
        self.pool_bytes[id(ws)] = self._ws_cost(info, kind)
        self.stats["workspaces_created"] += 1
        return ws

    def _evict_one(self, exclude) -> bool:
        """Frees one idle workspace other than `exclude`'s: a batched one if there is any."""
        for batched in (True, False):
            for key, lst in self.pool.items():
                if key != exclude and lst and (key[1] > 1) == batched:
                    ws = lst.pop()
                    self.used -= self.pool_bytes.pop(id(ws))
                    t0 = self.clock()
                    self.ex.destroy(ws)
                    self.stats["destroy_ms"] += (self.clock() - t0) * 1e3
                    self.stats["workspaces_evicted"] += 1
                    return True
        return False

    def _release(self, name: str, kind: int, ws):
        self.pool[(name, kind)].append(ws)

    def _learn(self, name: str, batched: bool, seconds):
        """Running mean (weight 1/4 for the newest) of a run's device time."""
        if seconds is None or seconds <= 0:
            return
        key = (name, batched)
        old = self.cost.get(key)
        self.cost[key] = seconds if old is None else 0.75 * old + 0.25 * seconds

    def _worth_batching(self, name: str, k: int) -> bool:
        """A batch of k is cheaper than k single runs (unknown until both have been timed)."""
        ts, tb = self.cost.get((name, False)), self.cost.get((name, True))
        return ts is None or tb is None or k * ts >= tb

    # ---- scheduling -------------------------------------------------------------------------
    def _admit(self):
        skipped = collections.deque()
        while self.pending and len(self.inflight) < self.max_inflight:
            q = self.pending.popleft()
            info = self.ex.info[q.graph]
            group = [q]
            cap = self._batch_cap(info) if info.batchable else 0
            if cap >= self.batch_min:
                same = [p for p in self.pending if p.graph == q.graph][: cap - 1]
                if len(same) + 1 >= self.batch_min and self._worth_batching(q.graph, len(same) + 1):
                    group += same
            k = len(group)
            ws = self._acquire(q.graph, k)
            if ws is None and k > 1:
                group, k = [q], 1      # no room for a batch: try the query on its own
                ws = self._acquire(q.graph, 1)
            if ws is None:
                if not self.inflight and not any(self.pool.values()):
                    need = self._ws_cost(info, 1) + self._out_cost(info, 1)
                    raise RuntimeError(f"query on {q.graph} needs {need} bytes; the budget is {self.budget}")
                skipped.append(q)      # memory is short for this graph: let other queries through
                continue
            for p in group[1:]:
                self.pending.remove(p)
            now = self.clock()
            for p in group:
                p.admitted = now
                p.batched = k > 1
            kind = 256 if k > 1 else 1
            out = self._out_cost(info, k)
            try:
                handle = self.ex.launch(ws, q.graph, [p.source for p in group])
            except Exception as exc:  # a failed launch answers its queries with the error
                self._fail(group, ws, kind, None, exc, out)
                continue
            self.inflight.append((handle, ws, q.graph, kind, group, out))
            self.stats["batches" if k > 1 else "singles"] += 1
        while skipped:
            self.pending.appendleft(skipped.pop())

    def _fail(self, group, ws, kind, handle, exc, out_bytes):
        """Answer `group` with an error and drop its workspace, whose state is unknown."""
        if handle is not None and hasattr(self.ex, "abandon"):
            self.ex.abandon(handle)
        cost = self.pool_bytes.pop(id(ws), 0)
        self.used -= cost + out_bytes
        try:
            self.ex.destroy(ws)
        except Exception:
            pass
        now = self.clock()
        for p in group:
            p.finished = now
            p.result = None
            p.error = f"{type(exc).__name__}: {exc}"
            self.done.append(p)
        self.stats["failed_queries"] += len(group)

    def _reap(self):
        still = []
        for item in self.inflight:
            handle, ws, name, kind, group, out = item
            try:
                if not self.ex.ready(handle):
                    still.append(item)
                    continue
                results = self.ex.collect(handle)
            except Exception as exc:
                self._fail(group, ws, kind, handle, exc, out)
                continue
            if hasattr(self.ex, "device_seconds"):
                self._learn(name, kind > 1, self.ex.device_seconds(handle))
            self.used -= out
            self._release(name, kind, ws)
            if results is None:
                # the batch overflowed: answer its queries one by one
                self.ex.info[name].batchable = False
                for p in reversed(group):
                    self.pending.appendleft(p)
                self.stats["batch_overflows"] += 1
                continue
            now = self.clock()
            for p, r in zip(group, results):
                p.finished = now
                p.result = r if self.keep_results else None
                self.done.append(p)
        self.inflight = still

    def run(self, queries: list[Query], idle_sleep: float = 0.0002) -> list[Query]:
        """Serve queries in arrival order; returns them with timings and results."""
        arrivals = collections.deque(sorted(queries, key=lambda q: q.arrival))
        t0 = self.clock()
        for q in arrivals:
            q.arrival += t0
        while arrivals or self.pending or self.inflight:
            now = self.clock()
            while arrivals and arrivals[0].arrival <= now:
                self.pending.append(arrivals.popleft())
            self._reap()
            self._admit()
            if not (arrivals and arrivals[0].arrival <= self.clock()):
                self.ex.idle(idle_sleep)
        for q in queries:
            q.arrival -= t0
            q.admitted -= t0
            q.finished -= t0
        return queries

    def close(self):
        for lst in self.pool.values():
            for ws in lst:
                self.ex.destroy(ws)
        self.pool.clear()
        self.used = 0


def poisson_queries(graph_names, nonisolated: dict, rate: float, count: int, seed: int = 1) -> list[Query]:
    """count queries with exponential inter-arrival times (mean 1/rate), graph uniform,
    source uniform among the graph's vertices of degree >= 1."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    names = list(graph_names)
    for i in range(count):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        g = names[rng.integers(len(names))]
        cand = nonisolated[g]
        out.append(Query(i, g, int(cand[rng.integers(len(cand))]), t))
    return out


def latency_summary(queries: list[Query]) -> dict:
    lat = np.array([q.latency for q in queries]) * 1e3
    span = max(q.finished for q in queries) - min(q.arrival for q in queries)
    return {"queries": len(queries), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "qps": len(queries) / span if span > 0 else float("inf"),
            "batched_fraction": float(np.mean([q.batched for q in queries]))}


# ---- GPU executor --------------------------------------------------------------------------------

class GpuExecutor:
    """Runs queries with libbfs on the current device, one stream per in-flight run."""

    def __init__(self, graphs: dict, max_inflight: int = 4):
        import torch

        from . import BFS_MODE_AUTO, Graph, Workspace, bfs_workspace_bytes

        self.torch = torch
        self.Workspace = Workspace
        self.mode = BFS_MODE_AUTO
        self.graphs = {}
        self.info = {}
        self.max_inflight = max_inflight
        self.streams = [torch.cuda.Stream() for _ in range(max_inflight)]
        self.free_streams = list(range(max_inflight))
        self.grid = None
        for name, g in graphs.items():
            G = Graph(g.offsets, g.cols)
            self.graphs[name] = G
            probe = Workspace(G)
            if self.grid is None:
                # persistent runs in flight together must fit on the GPU together: each of the
                # max_inflight streams gets an equal part of the device's co-resident workgroups
                self.grid = max(1, probe.grid_capacity() // max_inflight)
            nz = np.flatnonzero(np.diff(g.offsets))
            probe.run(int(nz[0]) if nz.size else 0, want_parent=False)
            probe.sync()
            ecc = probe.stats()["levels"] - 1
            probe.free()
            # a component's diameter is at most twice one vertex's eccentricity, and only
            # components of the probed vertex are bounded this way: batch graphs whose bound
            # fits a byte with a wide margin
            self.info[name] = GraphInfo(name, g.n, g.m, batchable=4 * ecc < 255,
                                        ws_bytes_single=bfs_workspace_bytes(G.handle, 1),
                                        ws_bytes_batch=bfs_workspace_bytes(G.handle, 256))

    def create(self, name, kind):
        from . import BFS_OPT_GRID, BFS_OPT_HOST_STATUS
        ws = self.Workspace(self.graphs[name], max_sources=kind)
        ws.set(BFS_OPT_GRID, self.grid)
        if kind == 1:  # single runs leave their device status where collect reads it without a wait
            ws.set(BFS_OPT_HOST_STATUS, 1)
        ws.name = name
        return ws

    def destroy(self, ws):
        ws.free()

    def launch(self, ws, name, sources):
        si = self.free_streams.pop()
        try:
            return self._launch(si, ws, name, sources)
        except Exception:
            self.free_streams.append(si)
            raise

    def _launch(self, si, ws, name, sources):
        torch = self.torch
        stream = self.streams[si]
        n = self.graphs[name].n
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            t0.record(stream)
            if len(sources) == 1:
                out = torch.empty(n, dtype=torch.int32, device="cuda")
                ws.run(sources[0], level=out, stream=stream, want_parent=False)
            else:
                out = torch.empty(n * len(sources), dtype=torch.uint8, device="cuda")
                ws.run_batch(sources, out, stream=stream)   # returns at once; overflow shows at sync
            t1.record(stream)
        return (si, ws, t0, t1, out, len(sources))

    def abandon(self, h):
        """Give back the stream of a run whose launch or collection failed."""
        si = h[0]
        if si not in self.free_streams:
            self.free_streams.append(si)

    def ready(self, h):
        return h[3].query()

    def device_seconds(self, h):
        """Device time of a completed run (its stream's events)."""
        return h[2].elapsed_time(h[3]) * 1e-3

    def collect(self, h):
        from . import BFSError, _lib
        torch = self.torch
        si, ws, t0, t1, out, k = h
        self.abandon(h)
        if k == 1:
            # the levels are complete in stream order; a host synchronisation per query would
            # also wait for whatever shares a hardware queue with the workspace's private stream,
            # so the run's device status comes from the copy it made before t1, without a wait
            st = ws.run_status()
            if st != _lib.BFS_OK:
                raise BFSError(st, "bfs_run", "device-side failure of a single run")
            return [out]
        try:
            ws.sync()            # a batch's overflow (and device-side failures) surface here
        except BFSError as e:
            if e.status != _lib.BFS_EOVERFLOW:
                raise
            return None          # a level did not fit in a byte: the scheduler re-queues the sources
        # converted on the run's own stream: `out` belongs to that stream's memory, which the
        # next run there may reuse as soon as this returns; the caller's stream then waits
        stream = self.streams[si]
        with torch.cuda.stream(stream):
            lv = out.view(-1, k).to(torch.int32)
            lv.masked_fill_(lv == 255, -1)
        cur = torch.cuda.current_stream()
        cur.wait_stream(stream)
        lv.record_stream(cur)
        return [lv[:, j] for j in range(k)]

    def idle(self, s):
        time.sleep(s)
