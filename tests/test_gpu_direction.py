"""Direction optimisation (bottom-up levels) gives the same levels and min-id
parents as the oracle, whether levels switch by the default rule or every
level is forced bottom-up."""
import numpy as np
import pytest

import graphgen as gg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import BFS_MODE_DIRECTION, Graph, Workspace  # noqa: E402
from tests.gpu_util import assert_same, run_single  # noqa: E402

FORCE = {"bu_alpha": 1 << 20, "bu_beta": 1 << 20}   # bottom-up at every level the frontier bits allow


@pytest.fixture(scope="module")
def graphs():
    out = {}
    for name, make in [("rmat16", lambda: gg.rmat(16, seed=61)), ("rmat18", lambda: gg.rmat(18, seed=62)),
                       ("er", lambda: gg.erdos_renyi(50000, 5.0, seed=63)), ("grid", lambda: gg.grid(120, 90)),
                       ("forest", lambda: gg.powerlaw_forest(40000, seed=64))]:
        g = make()
        out[name] = (g, Graph(g.offsets, g.cols))
    return out


@pytest.mark.parametrize("name", ["rmat16", "rmat18", "er", "grid", "forest"])
@pytest.mark.parametrize("opts", [{}, FORCE, dict(FORCE, small_edges=0), {"small_edges": 0, "grid": 7}],
                         ids=["rule", "forced", "forced-no-small", "rule-grid7"])
def test_direction_matches_oracle(graphs, name, opts):
    g, G = graphs[name]
    ws = Workspace(G, mode=BFS_MODE_DIRECTION, **opts)
    for s in gg.pick_sources(g, 2, seed=len(name) + len(opts)):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, int(s))
        if opts.get("small_edges") == 0 and "bu_alpha" in opts:
            assert ws.stats()["bottom_up_levels"] > 0


def test_rule_goes_bottom_up_on_rmat(graphs):
    g, G = graphs["rmat18"]
    ws = Workspace(G, mode=BFS_MODE_DIRECTION)
    s = gg.pick_sources(g, 1, seed=5)[0]
    lv, par = run_single(ws, s)
    assert_same(lv, par, g, int(s))
    assert ws.stats()["bottom_up_levels"] >= 1


def test_direction_levels_only_and_multiroot(graphs):
    g, G = graphs["rmat16"]
    ws = Workspace(G, mode=BFS_MODE_DIRECTION, **FORCE)
    s = gg.pick_sources(g, 1, seed=8)[0]
    lv, _ = run_single(ws, s, want_parent=False)
    assert_same(lv, None, g, int(s))
    roots = gg.pick_sources(g, 9, seed=2)
    lv, par = ws.run_multiroot(roots)
    ws.sync()
    assert_same(lv.cpu().numpy(), par.cpu().numpy(), g, roots)


def test_direction_with_hot_filter():
    g = gg.rmat(13, seed=66)
    G = Graph(g.offsets, g.cols, hot=True)
    for opts in ({}, FORCE, {"bu_alpha": 2, "bu_beta": 2, "grid": 3, "small_edges": 0}):
        ws = Workspace(G, mode=BFS_MODE_DIRECTION, **opts)
        for s in gg.pick_sources(g, 3, seed=4):
            lv, par = run_single(ws, s)
            assert_same(lv, par, g, int(s))


@pytest.mark.parametrize("name", ["rmat16", "rmat18", "er"])
def test_levels_handed_over_by_the_group_can_go_bottom_up(graphs, name):
    # forced bottom-up with group levels on: every level the group of workgroups does not run
    # goes bottom-up, the ones it hands over included (their frontier bits are rebuilt from the
    # handed-over queue)
    g, G = graphs[name]
    ws = Workspace(G, mode=BFS_MODE_DIRECTION, **FORCE)
    for s in gg.pick_sources(g, 3, seed=12):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, int(s))
        st = ws.stats()
        assert st["small_levels"] > 0 and st["bottom_up_levels"] > 0
        assert st["levels"] == st["small_levels"] + st["bottom_up_levels"], (int(s), st)
