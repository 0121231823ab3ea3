"""bfs_run_noalloc, the single-source search that allocates nothing, against
bfs_run on the same graphs: bit-exact levels and parents, on two calls in a
row (the second on a smaller graph, so it reuses scratch that a larger search
filled), with and without parents, and the size limit of its static scratch.
All calls go through the C ABI."""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import BFSError, Graph, Workspace, bfs_run_noalloc  # noqa: E402
from paper_2209_08764_amd import _lib  # noqa: E402


def _log(*a):
    print("[no_alloc]", *a, flush=True)


def _reference(G, s):
    ws = Workspace(G)
    lv, par = ws.run(s)
    ws.sync()
    out = lv.cpu().numpy(), par.cpu().numpy()
    ws.free()
    return out


def _noalloc(G, s, want_parent=True):
    lv = torch.full((G.n,), 7, dtype=torch.int32, device="cuda")
    par = torch.full((G.n,), 7, dtype=torch.int32, device="cuda") if want_parent else None
    st = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    bfs_run_noalloc(G.handle, s, lv, par, st)
    torch.cuda.synchronize()
    return lv.cpu().numpy(), (par.cpu().numpy() if want_parent else None), int(st.item())


def test_noalloc_matches_bfs_run_twice_second_smaller():
    big = gg.rmat(16, 16, seed=41)         # 2^16 vertices, ~1.8 M entries: several tiles per level
    small = gg.grid(70, 33)                # high diameter: group levels and a ragged tail
    cases = [(big, int(gg.pick_sources(big, 1, seed=42)[0])), (small, 5)]
    # the larger graph with the hot-vertex filter, so its scratch holds the hot-bit arrays too
    graphs = [Graph(big.offsets, big.cols, hot=True), Graph(small.offsets, small.cols)]
    for (g, s), G in zip(cases, graphs):
        _log(f"n={g.n} m={g.m} source={s}")
        want_l, want_p = _reference(G, s)
        ol, op = oracle.bfs(g.offsets, g.cols, s)
        assert np.array_equal(want_l, ol) and np.array_equal(want_p, op)
        got_l, got_p, st = _noalloc(G, s)
        assert st == _lib.BFS_OK
        assert np.array_equal(got_l, want_l)
        assert np.array_equal(got_p, want_p)
    # the same two graphs again, now without parents, then the larger one once more
    for (g, s), G in zip(cases + cases[:1], graphs + graphs[:1]):
        got_l, got_p, st = _noalloc(G, s, want_parent=False)
        assert st == _lib.BFS_OK and got_p is None
        assert np.array_equal(got_l, oracle.bfs(g.offsets, g.cols, s)[0])
    for G in graphs:
        G.free()


def test_noalloc_back_to_back_on_one_stream_without_sync():
    g = gg.rmat(14, 16, seed=43)
    G = Graph(g.offsets, g.cols)
    srcs = [int(x) for x in gg.pick_sources(g, 4, seed=44)]
    outs = []
    for s in srcs:
        lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
        par = torch.empty(g.n, dtype=torch.int32, device="cuda")
        bfs_run_noalloc(G.handle, s, lv, par)
        outs.append((lv, par))
    torch.cuda.synchronize()
    for s, (lv, par) in zip(srcs, outs):
        want_l, want_p = oracle.bfs(g.offsets, g.cols, s)
        assert np.array_equal(lv.cpu().numpy(), want_l)
        assert np.array_equal(par.cpu().numpy(), want_p)
    G.free()


def test_noalloc_rejects_a_graph_beyond_its_scratch():
    n = 3 << 20                            # 3 M isolated vertices: ~90 MB of search scratch
    G = Graph(np.zeros(n + 1, np.int32), np.zeros(0, np.int32))
    lv = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(BFSError) as e:
        bfs_run_noalloc(G.handle, 0, lv)
    assert e.value.status == _lib.BFS_ENOMEM
    assert "static scratch" in str(e.value)
    with pytest.raises(BFSError) as e:
        bfs_run_noalloc(G.handle, n, lv)
    assert e.value.status == _lib.BFS_ERANGE
    G.free()
