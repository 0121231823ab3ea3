"""The hot-vertex filter (LDS copy of the visited bits of the highest-degree
vertices) never changes a result: levels and min-id parents equal the oracle's
with and without it, on every mode and parent rule."""
import numpy as np
import pytest

import graphgen as gg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import (BFS_MODE_AUTO, BFS_MODE_INSENSITIVE, BFS_MODE_LEVEL, Graph,  # noqa: E402
                                  Workspace)
from tests.gpu_util import assert_same, run_single  # noqa: E402

HOT_MAX = 391168  # hot numbers the library hands out (LDS bits of the filter)


@pytest.fixture(scope="module")
def rmat18():
    g = gg.rmat(18, seed=181)
    return g, Graph(g.offsets, g.cols), Graph(g.offsets, g.cols, hot=False)


def test_size_rule_builds_filter(rmat18):
    g, G, lean = rmat18
    assert g.m >= 1 << 22
    # one word per edge, plus the id of each hot vertex (all of degree >= 1 here)
    hot = lambda h: min(HOT_MAX, int((np.diff(h.offsets) > 0).sum()))
    assert G.aux_bytes == 4 * (g.m + hot(g)) and lean.aux_bytes == 0
    small = gg.rmat(10, seed=1)
    assert Graph(small.offsets, small.cols).aux_bytes == 0
    assert Graph(small.offsets, small.cols, hot=True).aux_bytes == 4 * (small.m + hot(small))


@pytest.mark.parametrize("mode", [BFS_MODE_AUTO, BFS_MODE_LEVEL, BFS_MODE_INSENSITIVE])
@pytest.mark.parametrize("push", [0, 1 << 30, None])
def test_filter_matches_oracle(rmat18, mode, push):
    g, G, lean = rmat18
    opts = {} if push is None else {"push_edges": push}
    src = gg.pick_sources(g, 2, seed=mode * 7 + (push or 3))
    for graph in (G, lean):
        ws = Workspace(graph, mode=mode, **opts)
        for s in src:
            lv, par = run_single(ws, s)
            assert_same(lv, par, g, int(s))


@pytest.mark.parametrize("grid", [1, 3, 16])
def test_forced_filter_with_long_shares(grid):
    # few workgroups make every share long enough for the LDS copy; every vertex
    # of degree >= 1 is hot on a small graph
    for make in (lambda: gg.rmat(12, seed=5), lambda: gg.erdos_renyi(20000, 6.0, seed=3),
                 lambda: gg.grid(90, 70)):
        g = make()
        G = Graph(g.offsets, g.cols, hot=True)
        ws = Workspace(G, grid=grid, small_edges=0)
        for s in gg.pick_sources(g, 2, seed=grid):
            lv, par = run_single(ws, s)
            assert_same(lv, par, g, int(s))
        roots = gg.pick_sources(g, 5, seed=9)
        lv, par = ws.run_multiroot(roots)
        ws.sync()
        assert_same(lv.cpu().numpy(), par.cpu().numpy(), g, roots)


def test_more_hot_vertices_than_fit():
    # more vertices of degree >= 1 than hot numbers: only the top of the degree order is hot
    g = gg.erdos_renyi(500000, 3.0, seed=8)
    assert int((np.diff(g.offsets) > 0).sum()) > HOT_MAX
    G = Graph(g.offsets, g.cols, hot=True)
    ws = Workspace(G, grid=8, small_edges=0)
    for s in gg.pick_sources(g, 2, seed=1):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, int(s))
