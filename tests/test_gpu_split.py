"""GPU parity of the split ablation (BFS_OPT_SPLIT = 1): each share finds its
sub-tile start points by binary search of the degree prefix sums instead of
the paper's Find-StartExpPoint scatter.  Levels and parents must equal the
oracle's bit for bit in every mode that splits levels into shares, on graphs
whose levels span one to many thousands of sub-tiles, with ragged tails, the
hot-vertex filter and dense levels, multi-root runs and the per-level launches."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.gpu_util import assert_same, run_single

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import (BFS_MODE_AUTO, BFS_MODE_DIRECTION, BFS_MODE_INSENSITIVE,  # noqa: E402
                                  BFS_MODE_LEVEL, BFS_OPT_SPLIT, BFSError, Graph, Workspace)

SPLIT_MODES = [BFS_MODE_AUTO, BFS_MODE_LEVEL, BFS_MODE_INSENSITIVE, BFS_MODE_DIRECTION]


@pytest.mark.parametrize("mode", SPLIT_MODES)
@pytest.mark.parametrize("make,hot,small_edges", [
    (lambda: gg.rmat(14, seed=21), None, None),
    (lambda: gg.rmat(16, seed=23), True, None),          # hot-vertex filter, dense levels
    (lambda: gg.grid(64, 64), None, 0),                  # every level on the grid, shares of 1-2 sub-tiles
    (lambda: gg.grid(1, 3000), None, 0),                 # a path: 3000 levels of one edge pair
    (lambda: gg.erdos_renyi(1 << 15, 8.0, seed=4), None, None),
])
def test_search_split_matches_oracle(mode, make, hot, small_edges):
    g = make()
    G = Graph(g.offsets, g.cols, hot=hot)
    opts = {} if small_edges is None else {"small_edges": small_edges}
    ws = Workspace(G, mode=mode, split_search=1, **opts)
    for s in gg.pick_sources(g, 3, seed=mode + 7):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [s])


def test_search_split_at_the_default_grid():
    # R-MAT 18: ~7.6 M entries, a default grid of several hundred workgroups, levels of
    # thousands of sub-tiles per share
    g = gg.rmat(18, seed=31)
    G = Graph(g.offsets, g.cols)
    a = Workspace(G)
    b = Workspace(G, split_search=1)
    for s in gg.pick_sources(g, 3, seed=32):
        la, pa = run_single(a, s)
        lb, pb = run_single(b, s)
        want = assert_same(la, pa, g, [s])
        assert_same(lb, pb, g, [s], want=want)
    assert b.stats()["grid"] == a.stats()["grid"]


def test_search_split_multiroot():
    parts = [gg.rmat(9, seed=40 + i) for i in range(6)] + [gg.grid(20, 30), gg.powerlaw_forest(3000, seed=3)]
    u, base = gg.disjoint_union(parts)
    roots = np.array([int(base[i]) + int(gg.pick_sources(p, 1, seed=i)[0]) for i, p in enumerate(parts)], np.int32)
    ws = Workspace(Graph(u.offsets, u.cols), split_search=1)
    lv, par = ws.run_multiroot(roots)
    ws.sync()
    want_l, want_p = oracle.bfs(u.offsets, u.cols, roots)
    assert np.array_equal(lv.cpu().numpy(), want_l)
    assert np.array_equal(par.cpu().numpy(), want_p)


def test_split_option_is_checked():
    g = gg.grid(8, 8)
    ws = Workspace(Graph(g.offsets, g.cols))
    with pytest.raises(BFSError):
        ws.set(BFS_OPT_SPLIT, 2)
    ws.set(BFS_OPT_SPLIT, 1)
    ws.set(BFS_OPT_SPLIT, 0)
