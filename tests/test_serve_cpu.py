"""Scheduler logic of the serving loop on the CPU: a fake executor answers with the
oracle on a simulated clock (no GPU).  Checks admission by memory, continuous
batching, eviction and that every answer equals the oracle's."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_2209_08764_amd.serve import GraphInfo, Query, Scheduler, latency_summary, poisson_queries


class FakeExecutor:
    """Runs queries with the CPU oracle; a run of e edges takes e * 1 ns of simulated time."""

    def __init__(self, graphs, slots=4, batchable=None):
        self.now = 0.0
        self.graphs = graphs
        self.info = {}
        for name, g in graphs.items():
            b = batchable[name] if batchable else True
            self.info[name] = GraphInfo(name, g.n, g.m, b, ws_bytes_single=1000 + 20 * g.n,
                                        ws_bytes_batch=5000 + 100 * g.n)
        self.live = set()
        self.max_live = 0
        self.launched = []

    def clock(self):
        return self.now

    def idle(self, s):
        self.now += max(s, 1e-5)

    def create(self, name, kind):
        ws = (name, kind, object())
        self.live.add(ws)
        self.max_live = max(self.max_live, len(self.live))
        return ws

    def destroy(self, ws):
        self.live.remove(ws)

    def launch(self, ws, name, sources):
        g = self.graphs[name]
        res = [oracle.bfs_levels(g.offsets, g.cols, s) for s in sources]
        cost = 1e-9 * g.m * (1 + 0.1 * len(sources)) + 1e-5
        self.launched.append((name, len(sources)))
        return (self.now + cost, res)

    def ready(self, h):
        return self.now >= h[0]

    def collect(self, h):
        return h[1]


@pytest.fixture(scope="module")
def graphs():
    return {"a": gg.rmat(10, seed=1), "b": gg.grid(30, 20), "c": gg.powerlaw_forest(2000, seed=2)}


def _nonisolated(graphs):
    return {k: np.flatnonzero(np.diff(g.offsets)) for k, g in graphs.items()}


def test_every_answer_matches_the_oracle(graphs):
    ex = FakeExecutor(graphs, batchable={"a": True, "b": False, "c": True})
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_inflight=3, clock=ex.clock)
    qs = poisson_queries(graphs, _nonisolated(graphs), rate=2e5, count=300, seed=4)
    sch.run(qs)
    for q in qs:
        g = graphs[q.graph]
        assert np.array_equal(q.result, oracle.bfs_levels(g.offsets, g.cols, q.source))
        assert q.arrival <= q.admitted <= q.finished
    s = latency_summary(qs)
    assert s["queries"] == 300 and s["p99_ms"] >= s["p50_ms"] >= 0
    # the non-batchable graph never runs in a batch; the others do once queries pile up
    assert all(k == 1 for name, k in ex.launched if name == "b")
    assert any(k > 1 for name, k in ex.launched if name != "b")
    assert sch.stats["batches"] > 0


def test_budget_is_never_exceeded_and_small_budgets_serialise(graphs):
    ex = FakeExecutor(graphs)
    # room for the largest single-source workspace and its output, so not for every graph at once
    one = max(i.ws_bytes_single + 4 * i.n for i in ex.info.values())
    sch = Scheduler(ex, budget_bytes=one + 10, max_inflight=4, clock=ex.clock)
    qs = poisson_queries(graphs, _nonisolated(graphs), rate=0, count=60, seed=2)   # all at once
    orig_acquire = sch._acquire

    def checked(name, k):
        ws = orig_acquire(name, k)
        assert sch.used <= sch.budget
        return ws

    sch._acquire = checked
    sch.run(qs)
    assert all(q.result is not None for q in qs)
    assert sch.stats["workspaces_evicted"] > 0        # graphs took turns in the budget


def test_batch_size_is_capped(graphs):
    ex = FakeExecutor({"a": graphs["a"]})
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_inflight=2, batch_max=16, clock=ex.clock)
    qs = poisson_queries({"a": 0}, _nonisolated(graphs), rate=0, count=100, seed=1)
    sch.run(qs)
    assert max(k for _, k in ex.launched) == 16
    assert sum(k for _, k in ex.launched) == 100


def test_batches_stay_within_their_share_of_the_budget(graphs):
    ex = FakeExecutor({"a": graphs["a"]})
    info = ex.info["a"]
    budget = 2 * (info.ws_bytes_batch + 10 * info.n) + 1    # a batch may hold 10 sources
    sch = Scheduler(ex, budget_bytes=budget, max_inflight=2, clock=ex.clock)
    qs = poisson_queries({"a": 0}, _nonisolated(graphs), rate=0, count=100, seed=3)
    sch.run(qs)
    assert max(k for _, k in ex.launched) == 10
    assert sum(k for _, k in ex.launched) == 100
    assert all(q.result is not None for q in qs)


def test_results_can_be_dropped_once_delivered(graphs):
    ex = FakeExecutor(graphs)
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_inflight=3, clock=ex.clock, keep_results=False)
    qs = poisson_queries(graphs, _nonisolated(graphs), rate=2e5, count=100, seed=5)
    sch.run(qs)
    assert all(q.result is None and q.error is None and q.finished >= q.arrival for q in qs)
    assert sch.used == sum(sch.pool_bytes.values())   # no output is still charged


def test_queries_keep_arrival_order_within_a_graph(graphs):
    ex = FakeExecutor({"b": graphs["b"]}, batchable={"b": False})
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_inflight=1, clock=ex.clock)
    qs = [Query(i, "b", i, 0.0) for i in range(20)]
    sch.run(qs)
    adm = [q.admitted for q in qs]
    assert adm == sorted(adm)


class FailingExecutor(FakeExecutor):
    """Fails every launch on graph "b" and every collection of a batch on graph "c"."""

    def launch(self, ws, name, sources):
        if name == "b":
            raise RuntimeError("launch failed")
        return super().launch(ws, name, sources) + (name, len(sources))

    def ready(self, h):
        return self.now >= h[0]

    def collect(self, h):
        if h[2] == "c" and h[3] > 1:
            raise RuntimeError("device fault")
        return h[1]


def test_failed_requests_do_not_stop_the_loop(graphs):
    ex = FailingExecutor(graphs)
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_inflight=3, clock=ex.clock)
    qs = poisson_queries(graphs, _nonisolated(graphs), rate=2e5, count=200, seed=8)
    sch.run(qs)
    failed = [q for q in qs if q.error is not None]
    served = [q for q in qs if q.error is None]
    assert {q.graph for q in failed} <= {"b", "c"} and any(q.graph == "b" for q in failed)
    assert all(q.result is None for q in failed)
    assert sch.stats["failed_queries"] == len(failed)
    # every other query is answered, and correctly
    assert served and all(q.graph == "a" or (q.graph == "c" and not q.batched) for q in served)
    for q in served:
        g = graphs[q.graph]
        assert np.array_equal(q.result, oracle.bfs_levels(g.offsets, g.cols, q.source))
    # failed runs gave their workspaces back to the budget
    assert sch.used == sum(sch.pool_bytes.values())


def test_batches_use_free_budget_and_singles_evict_batches_first(graphs):
    ex = FakeExecutor(graphs)
    info = ex.info
    one_batch = max(i.ws_bytes_batch + 256 * i.n for i in info.values())
    singles = sum(i.ws_bytes_single + 4 * i.n for i in info.values())
    sch = Scheduler(ex, budget_bytes=singles + one_batch, max_inflight=2, clock=ex.clock, batch_share=1.0)
    orig_evict, orig_acquire = sch._evict_one, sch._acquire
    events = []

    def evict(exclude):
        idle_batched = sum(len(v) for key, v in sch.pool.items() if key[1] > 1 and key != exclude)
        kinds_before = {key: len(v) for key, v in sch.pool.items()}
        ok = orig_evict(exclude)
        gone = [key for key, v in sch.pool.items() if len(v) < kinds_before.get(key, 0)]
        events.append((idle_batched, gone))
        return ok

    def acquire(name, k):
        before = len(events)
        ws = orig_acquire(name, k)
        if k > 1:
            assert len(events) == before          # a batch never evicts
        return ws

    sch._evict_one, sch._acquire = evict, acquire
    qs = poisson_queries(graphs, _nonisolated(graphs), rate=5e4, count=400, seed=9)
    sch.run(qs)
    assert all(q.result is not None for q in qs)
    assert sch.used <= sch.budget and sch.stats["batches"] > 0
    for idle_batched, gone in events:
        if gone and gone[0][1] == 1:
            assert idle_batched == 0              # singles go only when no batched workspace is idle


class TimedExecutor(FakeExecutor):
    """Reports device time: a single run costs 1 unit, a batch 20 units whatever its size."""

    unit = 1e-4

    def launch(self, ws, name, sources):
        g = self.graphs[name]
        res = [oracle.bfs_levels(g.offsets, g.cols, s) for s in sources]
        cost = self.unit * (20 if len(sources) > 1 else 1)
        self.launched.append((name, len(sources)))
        return (self.now + cost, res, cost)

    def device_seconds(self, h):
        return h[2]



def test_batches_only_when_cheaper_than_single_runs(graphs):
    ex = TimedExecutor({"a": graphs["a"]})
    sch = Scheduler(ex, budget_bytes=10 ** 9, max_inflight=1, clock=ex.clock)
    srcs = _nonisolated(graphs)["a"]
    # a lone query (times a single run), a burst of 5 (no batch time yet: batched, and timed),
    # another 5 (5 singles cost less than a batch), then 30 (a batch costs less)
    waves = [(0.0, 1), (0.01, 5), (0.02, 5), (0.03, 30)]
    qs = []
    for t, count in waves:
        for _ in range(count):
            qs.append(Query(len(qs), "a", int(srcs[(7 * len(qs)) % len(srcs)]), t))
    sch.run(qs)
    for q in qs:
        assert np.array_equal(q.result, oracle.bfs_levels(graphs["a"].offsets, graphs["a"].cols, q.source))
    assert sch.cost[("a", False)] == pytest.approx(ex.unit)
    assert sch.cost[("a", True)] == pytest.approx(20 * ex.unit)
    assert [k for _, k in ex.launched] == [1, 5, 1, 1, 1, 1, 1, 30]
