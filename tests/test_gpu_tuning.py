"""The autotuner picks among valid settings, and results stay bit-exact under them."""
import json

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import Graph, Workspace, BFSError, _lib  # noqa: E402
from paper_2209_08764_amd.tuning import autotune  # noqa: E402


@pytest.fixture(scope="module")
def rmat12():
    g = gg.rmat(12, seed=77)
    return g, Graph(g.offsets, g.cols)


def test_batch_tuning_is_valid_and_exact(rmat12, tmp_path):
    g, G = rmat12
    ws = Workspace(G, max_sources=256)
    srcs = gg.pick_sources(g, 128, seed=2)
    cache = str(tmp_path / "tune.json")
    res = autotune(ws, srcs, cache=cache)
    assert not res["cached"]
    assert res["batch_grain"] in (512, 1024, 2048) and res["batch_tile"] in (1024, 2048, 4096)
    assert res["batch_levels"] in (2, 4, 8, 16)
    assert res["trials"] >= 1 + 8 + 5 + 3
    assert res["best_ms"] <= res["default_ms"]
    assert ws.tuning()["batch_grain"] == res["batch_grain"]
    out = ws.run_batch(srcs)
    ws.sync()
    want, ovf = oracle.bfs_batch_u8(g.offsets, g.cols, srcs)
    assert not ovf and np.array_equal(out.cpu().numpy().reshape(g.n, len(srcs)), want)
    # a new workspace takes the stored settings without timing
    ws2 = Workspace(G, max_sources=256)
    res2 = autotune(ws2, srcs, cache=cache)
    assert res2["cached"]
    for k in ("batch_grain", "batch_tile", "batch_levels", "batch_pull"):
        assert ws2.tuning()[k] == res[k]
    assert len(json.load(open(cache))) == 1


def test_single_tuning_is_valid_and_exact(rmat12):
    g, G = rmat12
    ws = Workspace(G)
    srcs = gg.pick_sources(g, 3, seed=4)
    res = autotune(ws, srcs, batch=False)
    assert res["small_edges"] in (0, 2048, 4096, 8192, 16384)
    assert res["grid"] >= 0 and res["push_edges"] > 0
    for s in srcs:
        lv, par = ws.run(int(s))
        ws.sync()
        wl, wp = oracle.bfs(g.offsets, g.cols, int(s))
        assert np.array_equal(lv.cpu().numpy(), wl) and np.array_equal(par.cpu().numpy(), wp)


def test_tuning_arguments_checked(rmat12):
    g, G = rmat12
    ws = Workspace(G, max_sources=8)
    with pytest.raises(BFSError) as e:
        autotune(ws, list(range(9)))
    assert e.value.status == _lib.BFS_EINVAL
    with pytest.raises(BFSError) as e:
        autotune(ws, [0, g.n])
    assert e.value.status == _lib.BFS_ERANGE
