"""GPU parity of the batched multi-source search against the oracle (bit-exact uint8 levels).

Column j of the [n][k] output must equal the single-source oracle's levels
from sources[j] mapped to uint8 (255 = unreached), for any mix of pushed and
pulled levels and any number of levels per graph replay.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import BFSError, Graph, Workspace, _lib  # noqa: E402


def _check(ws, g, srcs):
    out = ws.run_batch(srcs)
    ws.sync()
    got = out.cpu().numpy().reshape(g.n, len(srcs))
    want, ovf = oracle.bfs_batch_u8(g.offsets, g.cols, srcs)
    assert not ovf
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{len(bad)} entries differ, first (v, j) {bad[:5].tolist()}: " \
                          f"got {got[tuple(bad[0])]} want {want[tuple(bad[0])]}"


@pytest.fixture(scope="module")
def rmat13():
    g = gg.rmat(13, seed=31)
    return g, Graph(g.offsets, g.cols)


@pytest.mark.parametrize("k", [1, 7, 63, 64, 65, 130, 200, 256])
def test_batch_matches_oracle(rmat13, k):
    g, G = rmat13
    ws = Workspace(G, max_sources=256)
    _check(ws, g, gg.pick_sources(g, k, seed=k))


@pytest.mark.parametrize("pull", [-1, 0, 1000, 100000])
@pytest.mark.parametrize("levels", [1, 3, 8])
def test_push_pull_and_replay_length_do_not_change_results(rmat13, pull, levels):
    g, G = rmat13
    ws = Workspace(G, max_sources=256, batch_pull=pull, batch_levels=levels)
    _check(ws, g, gg.pick_sources(g, 96, seed=7))


@pytest.mark.parametrize("make", [lambda: gg.grid(40, 30), lambda: gg.powerlaw_forest(3000, seed=5),
                                  lambda: gg.erdos_renyi(5000, 3.0, seed=2), lambda: gg.rmat(11, seed=2, permute=False)])
def test_structured_graphs(make):
    g = make()
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G, max_sources=256)
    _check(ws, g, gg.pick_sources(g, 77, seed=3))


def test_duplicate_sources_and_reuse(rmat13):
    g, G = rmat13
    ws = Workspace(G, max_sources=128)
    s = gg.pick_sources(g, 20, seed=9)
    srcs = np.concatenate([s, s[:5], s[3:4]])
    _check(ws, g, srcs)
    _check(ws, g, s[:3])          # a different k: the captured loop is rebuilt
    _check(ws, g, srcs)


def test_overflow_on_long_paths():
    n = 300
    path = gg.from_edges(n, [(i, i + 1) for i in range(n - 1)])
    G = Graph(path.offsets, path.cols)
    ws = Workspace(G, max_sources=4)
    with pytest.raises(BFSError) as e:
        ws.run_batch([0, 10])
        ws.sync()                       # the run does not wait: bfs_sync reports the overflow
    assert e.value.status == _lib.BFS_EOVERFLOW
    # sources whose eccentricity fits are fine
    _check(ws, path, [150, 140])


def test_batch_errors(rmat13):
    g, G = rmat13
    ws = Workspace(G, max_sources=8)
    with pytest.raises(BFSError) as e:
        ws.run_batch(list(range(9)))
    assert e.value.status == _lib.BFS_EINVAL
    with pytest.raises(BFSError) as e:
        ws.run_batch([0, g.n])
    assert e.value.status == _lib.BFS_ERANGE
    single = Workspace(G)          # max_sources = 1 has no batched buffers
    with pytest.raises(BFSError):
        single.run_batch([1, 2])


@pytest.mark.parametrize("grain", [512, 1024, 2048])
@pytest.mark.parametrize("tile", [1024, 2048, 4096])
def test_every_launch_shape_matches_oracle(rmat13, grain, tile):
    g, G = rmat13
    ws = Workspace(G, max_sources=256, batch_grain=grain, batch_tile=tile)
    t = ws.tuning()
    assert (t["batch_grain"], t["batch_tile"]) == (grain, tile)
    _check(ws, g, gg.pick_sources(g, 150, seed=grain + tile))
    # a pull-only and a push-only pass with the same shape
    ws.set(_lib.BFS_OPT_BATCH_PULL, 0)
    _check(ws, g, gg.pick_sources(g, 40, seed=1))
    ws.set(_lib.BFS_OPT_BATCH_PULL, -1)
    _check(ws, g, gg.pick_sources(g, 40, seed=1))


@pytest.mark.parametrize("grain,tile", [(512, 4096), (2048, 1024)])
def test_launch_shapes_on_ragged_graphs(grain, tile):
    # n not a multiple of any tile, long rows cut by many sub-tiles, isolated vertices
    g, _ = gg.disjoint_union([gg.grid(37, 29), gg.rmat(10, seed=4), gg.powerlaw_forest(777, seed=9)])
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G, max_sources=256, batch_grain=grain, batch_tile=tile)
    _check(ws, g, gg.pick_sources(g, 255, seed=5))


def test_bad_launch_shape_rejected(rmat13):
    g, G = rmat13
    ws = Workspace(G, max_sources=4)
    for opt, val in [(_lib.BFS_OPT_BATCH_GRAIN, 768), (_lib.BFS_OPT_BATCH_TILE, 512)]:
        with pytest.raises(BFSError) as e:
            ws.set(opt, val)
        assert e.value.status == _lib.BFS_EINVAL
    single = Workspace(G)
    with pytest.raises(BFSError):
        single.set(_lib.BFS_OPT_BATCH_GRAIN, 512)


@pytest.mark.parametrize("pull", [0, 100000, -1])
@pytest.mark.parametrize("k", [64, 200, 256])
def test_hot_numbered_graph_pull_levels(pull, k):
    # with the hot-vertex numbering, pull levels gather hot neighbours' masks from the compact
    # copy refreshed before each pull level (hot vertices that are not active hold zero there)
    g = gg.rmat(14, seed=61)
    G = Graph(g.offsets, g.cols, hot=True)
    assert G.aux_bytes > 0
    ws = Workspace(G, max_sources=256, batch_pull=pull, batch_levels=3)
    _check(ws, g, gg.pick_sources(g, k, seed=pull + k))
    _check(ws, g, gg.pick_sources(g, k, seed=pull + k + 1))   # masks left by the previous batch


@pytest.mark.parametrize("replays", [0, 1, 2])
@pytest.mark.parametrize("levels", [1, 3])
def test_levels_left_by_the_replays_finish_on_one_workgroup(replays, levels):
    # fewer replays than levels: the one-workgroup finish runs the rest (all of them with
    # none), push and pull levels, hot masks and ragged update tiles included
    parts = [gg.rmat(11, seed=8), gg.grid(45, 23), gg.powerlaw_forest(1500, seed=6)]
    g, _ = gg.disjoint_union(parts)
    for hot in (False, True):
        G = Graph(g.offsets, g.cols, hot=hot)
        for pull in (-1, 0, 2000):
            ws = Workspace(G, max_sources=256, batch_levels=levels, batch_replays=replays, batch_pull=pull)
            _check(ws, g, gg.pick_sources(g, 129, seed=replays + 10 * levels))
            assert ws.stats()["levels"] > replays * levels


def test_overflow_found_by_the_finish():
    n = 300
    path = gg.from_edges(n, [(i, i + 1) for i in range(n - 1)])
    ws = Workspace(Graph(path.offsets, path.cols), max_sources=4, batch_replays=1)
    with pytest.raises(BFSError) as e:
        ws.run_batch([0, 10])
        ws.sync()
    assert e.value.status == _lib.BFS_EOVERFLOW
    _check(ws, path, [150, 140])


def test_batched_run_returns_before_the_device_finishes():
    # R-MAT 20 with 256 sources takes milliseconds on the device; the call only enqueues
    g = gg.rmat(20, seed=77)
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G, max_sources=256)
    srcs = gg.pick_sources(g, 256, seed=4)
    level = torch.empty(g.n * 256, dtype=torch.uint8, device="cuda")
    ws.run_batch(srcs, level)
    ws.sync()                           # learns the depth, so the next run enqueues no extra replay
    pending = []
    for _ in range(3):
        ws.run_batch(srcs, level)
        ev = torch.cuda.Event()
        ev.record()
        pending.append(not ev.query())  # the device is still searching when the call returns
        ws.sync()
    assert all(pending)
    got = level.cpu().numpy().reshape(g.n, 256)
    for j in (0, 101, 255):
        want = oracle.bfs_levels(g.offsets, g.cols, int(srcs[j]))
        want8 = np.where(want < 0, 255, want).astype(np.uint8)
        assert np.array_equal(got[:, j], want8)


def test_batched_runs_queued_back_to_back_keep_their_own_arguments(rmat13):
    # two batched runs on one stream with no synchronisation between them, different k and
    # outputs: each run's arguments travel with its own launch
    g, G = rmat13
    ws = Workspace(G, max_sources=256)
    a = gg.pick_sources(g, 200, seed=21)
    b = gg.pick_sources(g, 37, seed=22)
    out_a = ws.run_batch(a)
    out_b = ws.run_batch(b)
    ws.sync()
    for out, srcs in ((out_a, a), (out_b, b)):
        got = out.cpu().numpy().reshape(g.n, len(srcs))
        want, ovf = oracle.bfs_batch_u8(g.offsets, g.cols, srcs)
        assert not ovf and np.array_equal(got, want)


@pytest.mark.parametrize("pull", [-1, 0, None])
def test_smaller_batches_after_a_full_one(pull):
    # a batch of 256 sources fills all four mask words of every vertex it reaches; later batches
    # with fewer words (100 sources: 2, 40: 1) on the same workspace read those words as part of
    # each 32-byte gather but never use them
    g = gg.rmat(14, seed=67)
    G = Graph(g.offsets, g.cols, hot=True)
    opts = {} if pull is None else {"batch_pull": pull}
    ws = Workspace(G, max_sources=256, **opts)
    for k in (256, 100, 40, 256, 1):
        _check(ws, g, gg.pick_sources(g, k, seed=300 + k))
