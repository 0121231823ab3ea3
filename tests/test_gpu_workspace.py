"""Workspaces on the GPU: a workspace starts with private queues for the
default options (levels of up to m / 24 edges keep queues, larger ones are
dense) and grows them when a run's mode, options or roots need more.  One
workspace then runs every such configuration in turn, each bit-exact.  A
workspace still in flight refuses a run from another stream (BFS_EBUSY)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.gpu_util import assert_same, run_single

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import (BFS_MODE_AUTO, BFS_MODE_DIRECTION, BFS_MODE_INSENSITIVE,  # noqa: E402
                                  BFS_MODE_LEVEL, BFS_OPT_DENSE_EDGES, BFS_OPT_MODE, BFS_OPT_PUSH_EDGES,
                                  BFS_OPT_SMALL_EDGES, Graph, Workspace, bfs_workspace_bytes)


def test_default_workspace_is_sized_for_dense_levels():
    g = gg.rmat(16, seed=51)
    G = Graph(g.offsets, g.cols)
    b = bfs_workspace_bytes(G.handle, 1)
    # per-vertex arrays (32.5 B per vertex with the roots), statistics (2 MiB) and queues for a
    # 24th of the edges
    assert b < 32.5 * g.n + g.m / 24 * 4 + 4 * 2048 * 4 + (3 << 20)
    assert b > 32 * g.n + g.m / 24 * 4


def test_one_workspace_grows_through_every_configuration():
    g = gg.rmat(15, seed=52)
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G)
    srcs = [int(x) for x in gg.pick_sources(g, 2, seed=53)]
    steps = [
        {BFS_OPT_MODE: BFS_MODE_AUTO},
        {BFS_OPT_DENSE_EDGES: 0},                               # every level keeps queues
        {BFS_OPT_DENSE_EDGES: g.m // 24, BFS_OPT_PUSH_EDGES: g.m},  # every level pushes with queues
        {BFS_OPT_PUSH_EDGES: g.m // 24, BFS_OPT_MODE: BFS_MODE_DIRECTION},
        {BFS_OPT_MODE: BFS_MODE_LEVEL},
        {BFS_OPT_MODE: BFS_MODE_INSENSITIVE, BFS_OPT_SMALL_EDGES: 1 << 30},
        {BFS_OPT_MODE: BFS_MODE_AUTO, BFS_OPT_SMALL_EDGES: 4096},
    ]
    for opts in steps:
        for k, v in opts.items():
            ws.set(k, v)
        for s in srcs:
            lv, par = run_single(ws, s)
            assert_same(lv, par, g, [s])
    # every vertex a root: the roots' queues span the whole vertex set
    roots = np.arange(g.n, dtype=np.int32)
    lv, par = ws.run_multiroot(roots)
    ws.sync()
    assert np.all(lv.cpu().numpy() == 0) and np.array_equal(par.cpu().numpy(), roots)
    some = roots[::97]
    lv, par = ws.run_multiroot(some)
    ws.sync()
    want_l, want_p = oracle.bfs(g.offsets, g.cols, some)
    assert np.array_equal(lv.cpu().numpy(), want_l) and np.array_equal(par.cpu().numpy(), want_p)


def test_create_and_free_wait_for_nothing_else_on_the_device():
    # a search of tens of milliseconds runs on another stream while a workspace is dropped and
    # another made: neither waits for it, and the new workspace still answers correctly
    import time
    big = gg.grid(2048, 2048)
    long_ws = Workspace(Graph(big.offsets, big.cols))
    g = gg.rmat(14, seed=5)
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G)
    src = int(gg.pick_sources(g, 1, seed=6)[0])
    run_single(ws, src)
    lv_big = torch.empty(big.n, dtype=torch.int32, device="cuda")
    other = torch.cuda.Stream()
    long_ws.run(0, level=lv_big, stream=other, want_parent=False)   # warm-up
    long_ws.sync()
    long_ws.run(0, level=lv_big, stream=other, want_parent=False)
    t0 = time.perf_counter()
    ws.free()
    t1 = time.perf_counter()
    ws2 = Workspace(G)
    t2 = time.perf_counter()
    done = torch.cuda.Event()
    done.record(other)
    still_running = not done.query()
    assert still_running, "the long search ended before the measurement; it proves nothing"
    assert t1 - t0 < 0.010 and t2 - t1 < 0.010, (t1 - t0, t2 - t1)
    lv, par = run_single(ws2, src)
    assert_same(lv, par, g, [src])
    long_ws.sync()


def test_run_from_another_stream_while_in_flight_is_refused():
    # a search of the 2048 x 2048 grid (4095 levels) runs for tens of milliseconds; the
    # workspace refuses a run from another stream until it has finished, accepts one on the
    # same stream (stream order), and afterwards accepts any stream
    from paper_2209_08764_amd import BFSError, _lib, bfs_run
    g = gg.grid(2048, 2048)
    ws = Workspace(Graph(g.offsets, g.cols))
    level = torch.empty(g.n, dtype=torch.int32, device="cuda")
    parent = torch.empty_like(level)
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    bfs_run(ws.handle, 0, level, parent, stream=a)
    with pytest.raises(BFSError) as err:
        bfs_run(ws.handle, 0, level, parent, stream=b)
    assert err.value.status == _lib.BFS_EBUSY
    bfs_run(ws.handle, 0, level, parent, stream=a)        # same stream: queued behind the first
    a.synchronize()
    bfs_run(ws.handle, g.n - 1, level, parent, stream=b)
    b.synchronize()
    ws.sync()
    assert ws.stats()["status"] == 0
    lv = level.cpu().numpy()
    assert lv[0] == 2 * 2047 and lv[g.n - 1] == 0
