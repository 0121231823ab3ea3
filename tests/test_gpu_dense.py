"""Dense levels (frontier kept as bits, linearised in vertex order) against the CPU oracle.

A pull level with at least BFS_OPT_DENSE_EDGES edges records its new
vertices in the frontier bitmap instead of private queues and compacts them
by vertex range.  These cases force that path on every eligible level
(threshold 1), switch it off (0), and cross it with the parent rules,
group levels, grid sizes, multi-root runs, isolated vertices and
level-only runs: levels and min-id parents stay bit-exact.
"""
import numpy as np
import pytest

import graphgen as gg
from tests.gpu_util import assert_same, run_single

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import (BFS_MODE_AUTO, BFS_MODE_INSENSITIVE, BFS_OPT_DENSE_EDGES, BFSError,  # noqa: E402
                                  Graph, Workspace, bfs_workspace_set_option)

GRAPHS = {
    "rmat15": lambda: gg.rmat(15, seed=151),
    "er": lambda: gg.erdos_renyi(60000, 7.0, seed=12),
    "grid": lambda: gg.grid(300, 200),
    "forest": lambda: gg.powerlaw_forest(50000, nroots=40, seed=3),   # isolated trees, unreached parts
}


@pytest.fixture(scope="module", params=sorted(GRAPHS))
def graph(request):
    g = GRAPHS[request.param]()
    return g, Graph(g.offsets, g.cols)


@pytest.mark.parametrize("dense", [1, 0, None])
@pytest.mark.parametrize("push", [0, None])
def test_dense_levels_match_oracle(graph, dense, push):
    g, G = graph
    opts = {}
    if dense is not None:
        opts["dense_edges"] = dense
    if push is not None:
        opts["push_edges"] = push
    ws = Workspace(G, **opts)
    for s in gg.pick_sources(g, 3, seed=(dense or 5) + (push or 7)):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [int(s)])


@pytest.mark.parametrize("grid", [1, 3, 16, 0])
@pytest.mark.parametrize("small_edges", [0, None])
def test_dense_levels_any_grid(graph, grid, small_edges):
    g, G = graph
    opts = {"dense_edges": 1, "push_edges": 0, "grid": grid}
    if small_edges is not None:
        opts["small_edges"] = small_edges
    ws = Workspace(G, **opts)
    s = int(gg.pick_sources(g, 1, seed=grid + 3)[0])
    lv, par = run_single(ws, s)
    assert_same(lv, par, g, [s])


def test_dense_levels_without_parents(graph):
    # no parents to find: every level with enough edges is dense, push levels included
    g, G = graph
    ws = Workspace(G, dense_edges=1)
    for s in gg.pick_sources(g, 2, seed=41):
        lv, _ = run_single(ws, s, want_parent=False)
        assert_same(lv, None, g, [int(s)])


def test_dense_levels_multiroot_and_insensitive(graph):
    g, G = graph
    roots = gg.pick_sources(g, 9, seed=77)
    for mode in (BFS_MODE_AUTO, BFS_MODE_INSENSITIVE):
        ws = Workspace(G, mode=mode, dense_edges=1, push_edges=0)
        lv, par = ws.run_multiroot(roots)
        ws.sync()
        assert_same(lv.cpu().numpy(), par.cpu().numpy(), g, roots)


def test_dense_repeated_runs_reuse_bits():
    # back-to-back searches from different sources on one workspace: the frontier bits a
    # dense level leaves behind never leak into the next search
    g = gg.rmat(14, seed=9)
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G, dense_edges=1, push_edges=0)
    for s in gg.pick_sources(g, 6, seed=2):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [int(s)])
        lv, _ = run_single(ws, s, want_parent=False)
        assert_same(lv, None, g, [int(s)])


def test_dense_threshold_rejects_negative():
    g = gg.rmat(8, seed=1)
    ws = Workspace(Graph(g.offsets, g.cols))
    with pytest.raises(BFSError):
        bfs_workspace_set_option(ws.handle, BFS_OPT_DENSE_EDGES, -1)
    assert ws.tuning()["dense_edges"] == max(g.m // 24, 1)
    bfs_workspace_set_option(ws.handle, BFS_OPT_DENSE_EDGES, 0)
    assert ws.tuning()["dense_edges"] == 0


def late_parent_graph(k: int = 6000, fillers: int = 3000, f: int = 64, seed: int = 9):
    """New vertices whose only level-l neighbours sit late in their sorted rows.

    The source (the largest id) reaches f frontier vertices with the next-largest ids;
    each of the k vertices 0..k-1 joins one or two of them and r distinct filler vertices
    whose ids lie between, so its first level-1 neighbour is at row position r.  r takes
    values on both sides of every scan boundary (2, 34, 34 + 64 * j) up to 600, so a
    parent pull meets rows found at once, rows a lane finishes, and rows scanned 64 at a
    time; all k vertices are new at level 2 and fill whole 2048-vertex chunks.
    """
    rng = np.random.default_rng(seed)
    n = k + fillers + f + 1
    s = n - 1
    fr = np.arange(n - 1 - f, n - 1)
    r_vals = np.array([0, 1, 2, 3, 5, 8, 20, 31, 33, 34, 35, 36, 40, 64, 97, 98, 99, 100, 161, 162, 300, 600])
    src, dst = [np.full(f, s)], [fr]
    for x in range(k):
        r = int(r_vals[x % r_vals.size]) if x % 5 else int(rng.integers(0, 40))
        par = rng.choice(fr, size=1 + (x % 2), replace=False)
        fill = k + rng.choice(fillers, size=r, replace=False)
        nb = np.concatenate([par, fill])
        src.append(np.full(nb.size, x))
        dst.append(nb)
    g = gg.csr_from_pairs(n, np.concatenate(src), np.concatenate(dst), name="late_parents")
    return g, s


@pytest.mark.parametrize("dense", [1, 0])
@pytest.mark.parametrize("grid", [0, 1, 5])
def test_parents_found_late_in_long_rows(dense, grid):
    g, s = late_parent_graph()
    # every level a grid level that pulls its parents
    ws = Workspace(Graph(g.offsets, g.cols), dense_edges=dense, push_edges=0, small_edges=0, grid=grid)
    lv, par = run_single(ws, s)
    want = assert_same(lv, par, g, [s])
    assert int((want[0] == 2).sum()) == 6000
