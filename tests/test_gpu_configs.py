"""Bit-exact parity on the five benchmark workloads at their full size.

Each workload is built exactly as graphgen.workloads builds it for bench.py
(same generators, seeds and sources) and every output element is compared
with the CPU oracle, run on host threads:

  C1  R-MAT scale 16, its seeded source: level and parent, every mode
  C2  4096 x 4096 grid from vertex 0: all 16.8 M levels and parents against
      the closed form (level = r + c, parent = the vertex above, else the
      one to the left) and against the oracle
  C3  R-MAT scale 24 at the library's default grid (512 workgroups on an
      MI355X): 8 of the 64 sources, level and parent, top-down and
      direction-optimising, plus the O(n + m) certificate of one of them
  C4  R-MAT scale 22, the 256 sources in one batched run, with the launch
      shape the autotuner picks on this graph and with the default shape,
      against the oracle's uint8 levels
  C5  the eight resident serving graphs: a Poisson mix of queries under a
      2 GB admission budget, each answer equal to its answer alone and,
      for a sample, to the oracle's
"""
import numpy as np
import pytest

import graphgen as gg
from graphgen import workloads as W
from oracle.certify import certify
from tests.gpu_util import assert_same, oracle_batch_u8, oracle_many, run_single

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

from paper_2209_08764_amd import (BFS_MODE_AUTO, BFS_MODE_DIRECTION, BFS_MODE_INSENSITIVE,  # noqa: E402
                                  BFS_MODE_LEVEL, Graph, Workspace)


def _log(*a):
    print("[configs]", *a, flush=True)


# ---- C1 ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [BFS_MODE_AUTO, BFS_MODE_DIRECTION, BFS_MODE_LEVEL, BFS_MODE_INSENSITIVE])
def test_c1_rmat16(mode):
    g, srcs = W.c1_rmat16()
    s = int(srcs[0])
    want = oracle_many(g, [s])[0]
    ws = Workspace(Graph(g.offsets, g.cols), mode=mode)
    lv, par = run_single(ws, s)
    assert_same(lv, par, g, [s], want=want)
    assert ws.stats()["levels"] == int(want[0].max()) + 1


# ---- C2 ----------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c2():
    g, srcs = W.c2_grid4096()
    Wd = 4096
    r, c = np.divmod(np.arange(g.n, dtype=np.int64), Wd)
    level = (r + c).astype(np.int32)
    parent = np.where(r > 0, (r - 1) * Wd + c, c - 1).astype(np.int32)
    parent[0] = 0
    return g, int(srcs[0]), (level, parent), Graph(g.offsets, g.cols)


def test_c2_closed_form_is_the_oracle(c2):
    g, s, closed, _ = c2
    want = oracle_many(g, [s])[0]
    np.testing.assert_array_equal(want[0], closed[0])
    np.testing.assert_array_equal(want[1], closed[1])


@pytest.mark.parametrize("mode", [BFS_MODE_AUTO, BFS_MODE_INSENSITIVE, BFS_MODE_DIRECTION])
def test_c2_grid4096(c2, mode):
    g, s, closed, G = c2
    ws = Workspace(G, mode=mode)
    lv, par = run_single(ws, s)
    assert_same(lv, par, g, [s], want=closed)
    st = ws.stats()
    assert st["levels"] == 8191 and st["status"] == 0


# ---- C3 ----------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c3():
    _log("C3: generating R-MAT scale 24")
    g, srcs = W.c3_rmat24()
    sub = [int(x) for x in srcs[:8]]
    _log(f"C3: n={g.n} m={g.m}; oracle on {len(sub)} sources")
    want = oracle_many(g, sub)
    _log("C3: oracle done")
    return g, sub, want, Graph(g.offsets, g.cols)


def test_c3_rmat24_default_grid(c3):
    g, sub, want, G = c3
    ws = Workspace(G)
    cap = torch.cuda.get_device_properties(0).multi_processor_count
    for s, w in zip(sub, want):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [s], want=w)
        st = ws.stats()
        assert st["status"] == 0
        # the graph is large enough for the default grid to be the co-resident maximum
        assert st["grid"] >= cap, st
        _log(f"C3 source {s}: {st['levels']} levels, grid {st['grid']}, bit-exact")


def test_c3_rmat24_direction(c3):
    g, sub, want, G = c3
    ws = Workspace(G, mode=BFS_MODE_DIRECTION)
    for s, w in zip(sub, want):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [s], want=w)
        assert ws.stats()["bottom_up_levels"] > 0


def test_c3_certificate(c3):
    g, sub, want, G = c3
    ws = Workspace(G)
    lv, par = run_single(ws, sub[0])
    _log("C3: certificate of one search")
    assert certify(g.offsets, g.cols, [sub[0]], lv, par) == []


# ---- C4 ----------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c4():
    _log("C4: generating R-MAT scale 22")
    g, srcs = W.c4_rmat22()
    _log(f"C4: n={g.n} m={g.m}; oracle on {len(srcs)} sources")
    want, ovf = oracle_batch_u8(g, srcs)
    assert not ovf
    _log("C4: oracle done")
    return g, srcs, want, Graph(g.offsets, g.cols)


@pytest.mark.parametrize("shape", ["default", "tuned"])
def test_c4_rmat22_256_batched(c4, shape):
    g, srcs, want, G = c4
    ws = Workspace(G, max_sources=256)
    if shape == "tuned":
        tune = ws.autotune(srcs, batch=True)
        _log(f"C4 tuned shape: {tune}")
    out = ws.run_batch(srcs)
    ws.sync()
    got = out.cpu().numpy().reshape(g.n, len(srcs))
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} entries differ, first {bad[:5].tolist()}"
    assert ws.stats()["status"] == 0


# ---- C5 ----------------------------------------------------------------------------------------

def test_c5_serving_graphs_mix_alone_oracle():
    from paper_2209_08764_amd.serve import GpuExecutor, Scheduler, latency_summary, poisson_queries
    _log("C5: generating the eight serving graphs")
    graphs = W.c5_graphs()
    ex = GpuExecutor(graphs, max_inflight=4)
    noniso = {k: np.flatnonzero(np.diff(g.offsets)) for k, g in graphs.items()}
    qs = poisson_queries(graphs, noniso, rate=2000.0, count=160, seed=21)
    sch = Scheduler(ex, budget_bytes=2_000_000_000, max_inflight=4)
    sch.run(qs)
    torch.cuda.synchronize()
    assert not any(q.error for q in qs)
    assert sch.stats["batches"] > 0 and sch.stats["singles"] > 0
    _log(f"C5: {latency_summary(qs)} {dict(sch.stats)}")
    # every answer equals the same query run alone
    wss = {}
    for q in qs:
        if q.graph not in wss:
            wss[q.graph] = Workspace(ex.graphs[q.graph])
        alone, _ = run_single(wss[q.graph], q.source, want_parent=False)
        got = q.result.cpu().numpy()
        assert np.array_equal(got, alone), (q.qid, q.graph, q.source, q.batched)
    # and a sample of them equals the oracle
    sample = qs[::5]
    by_graph = {}
    for q in sample:
        by_graph.setdefault(q.graph, []).append(q)
    for name, group in by_graph.items():
        g = graphs[name]
        wants = oracle_many(g, [q.source for q in group], with_parent=False)
        for q, w in zip(group, wants):
            assert np.array_equal(q.result.cpu().numpy(), w), (q.qid, name, q.source)
    sch.close()
