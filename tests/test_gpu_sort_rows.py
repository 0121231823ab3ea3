"""BFS_SORT_ROWS: a graph given with unsorted rows is searched as if its rows
were sorted (a device segmented sort into a copy the library owns): levels
and parents equal the oracle's, the caller's arrays are left as they were,
and BFS_VALIDATE accepts the unsorted input only together with the flag."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.gpu_util import assert_same, run_single

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import BFSError, Graph, Workspace, _lib  # noqa: E402


def _shuffled_rows(g, seed):
    rng = np.random.default_rng(seed)
    cols = g.cols.copy()
    for v in range(g.n):
        a, b = g.offsets[v], g.offsets[v + 1]
        if b - a > 1:
            cols[a:b] = rng.permutation(cols[a:b])
    return cols


@pytest.mark.parametrize("copy", [False, True])     # device arrays borrowed / host arrays copied
@pytest.mark.parametrize("hot", [None, True])
def test_unsorted_rows_are_sorted_by_the_library(copy, hot):
    g = gg.rmat(13, seed=71)
    unsorted = _shuffled_rows(g, 72)
    assert not np.array_equal(unsorted, g.cols)
    G = Graph(g.offsets, unsorted, copy=copy, validate=True, sort_rows=True, hot=hot)
    ws = Workspace(G)
    for s in gg.pick_sources(g, 4, seed=73):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [s])
    if not copy:
        # the borrowed arrays are the caller's, unchanged
        assert np.array_equal(G.cols.cpu().numpy(), unsorted)
    # the batched search on the same graph
    wb = Workspace(G, max_sources=64)
    srcs = gg.pick_sources(g, 64, seed=74)
    out = wb.run_batch(srcs)
    wb.sync()
    want, _ = oracle.bfs_batch_u8(g.offsets, g.cols, srcs)
    assert np.array_equal(out.cpu().numpy().reshape(g.n, 64), want)


def test_validate_rejects_unsorted_rows_without_the_flag():
    g = gg.rmat(10, seed=75)
    unsorted = _shuffled_rows(g, 76)
    with pytest.raises(BFSError) as e:
        Graph(g.offsets, unsorted, validate=True)
    assert e.value.status == _lib.BFS_EBADCSR
    Graph(g.offsets, unsorted, validate=True, sort_rows=True).free()
