"""GPU parity of single-source and multi-root search against the CPU oracle (bit-exact).

Every case calls the HIP library through its C ABI (via the ctypes binding)
and compares level and parent arrays element by element with oracle.bfs on
the same seeded graph.  Sizes span many shares of 2048 edges and ragged
tails; the mode/threshold/grid sweeps check that the benign race of the
owner de-duplication never changes a result.
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle.certify import certify
from tests.gpu_util import assert_same, run_single

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import (BFS_MODE_AUTO, BFS_MODE_INSENSITIVE, BFS_MODE_LEVEL,  # noqa: E402
                                  BFS_MODE_PLAIN, BFS_OPT_GRID, BFS_OPT_MODE, BFS_OPT_SMALL_EDGES, BFSError,
                                  Graph, Workspace, _lib)

MODES = [BFS_MODE_AUTO, BFS_MODE_LEVEL, BFS_MODE_PLAIN, BFS_MODE_INSENSITIVE]


@pytest.fixture(scope="module")
def rmat14():
    g = gg.rmat(14, seed=21)
    return g, Graph(g.offsets, g.cols)


def test_library_is_the_in_tree_build():
    lib = _lib.load()
    assert lib._name.endswith("paper_2209_08764_amd/libbfs.so")


@pytest.mark.parametrize("mode", MODES)
def test_rmat14_all_modes(rmat14, mode):
    g, G = rmat14
    ws = Workspace(G, mode=mode)
    for s in gg.pick_sources(g, 4, seed=mode + 1):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [s])


@pytest.mark.parametrize("small_edges", [0, 1, 100, 5000, 1 << 30])
@pytest.mark.parametrize("grid", [0, 1, 3, 37])
def test_thresholds_and_grids_do_not_change_results(rmat14, small_edges, grid):
    g, G = rmat14
    ws = Workspace(G, small_edges=small_edges, grid=grid)
    s = int(gg.pick_sources(g, 1, seed=5)[0])
    lv, par = run_single(ws, s)
    assert_same(lv, par, g, [s])


@pytest.mark.parametrize("make,srcs", [
    (lambda: gg.grid(64, 64), [0, 2080, 4095]),
    (lambda: gg.grid(257, 3), [0, 400]),
    (lambda: gg.grid(1, 3000), [0, 1500]),           # a path: 3000 levels
    (lambda: gg.powerlaw_forest(1 << 13, seed=3), None),
    (lambda: gg.erdos_renyi(1 << 14, 8.0, seed=4), None),
    (lambda: gg.rmat(10, seed=2, permute=False), None),
])
@pytest.mark.parametrize("mode", [BFS_MODE_AUTO, BFS_MODE_INSENSITIVE, BFS_MODE_LEVEL])
def test_structured_graphs(make, srcs, mode):
    g = make()
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G, mode=mode)
    if srcs is None:
        srcs = gg.pick_sources(g, 3, seed=9)
    for s in srcs:
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [s])


def _gen_petersen(n, k):
    return gg.from_edges(2 * n, [(i, (i + 1) % n) for i in range(n)] + [(i, n + i) for i in range(n)]
                         + [(n + i, n + (i + k) % n) for i in range(n)])


def _hypercube(d):
    return gg.from_edges(1 << d, [(v, v ^ (1 << b)) for v in range(1 << d) for b in range(d) if v < v ^ (1 << b)])


@pytest.mark.parametrize("mode", MODES)
def test_distance_regular_graphs_every_source(mode):
    # level counts fixed by the graph (Petersen 1,3,6; dodecahedron and Desargues 1,3,6,6,3,1;
    # Q_7 binomials), and levels and parents equal to the oracle's, from every vertex
    cases = [(_gen_petersen(5, 2), [1, 3, 6]), (_gen_petersen(10, 2), [1, 3, 6, 6, 3, 1]),
             (_gen_petersen(10, 3), [1, 3, 6, 6, 3, 1]), (_hypercube(7), [math.comb(7, i) for i in range(8)])]
    for g, counts in cases:
        ws = Workspace(Graph(g.offsets, g.cols), mode=mode)
        for s in range(g.n):
            lv, par = run_single(ws, s)
            assert np.bincount(lv).tolist() == counts, (g.n, s)
            assert_same(lv, par, g, [s])


@pytest.mark.parametrize("small_edges", [0, None])
def test_hypercube_closed_form(small_edges):
    # Q_12 (4096 vertices, 24576 directed edges, middle levels over 10 000 edges): level is the
    # Hamming distance; the min-id closer neighbour clears the highest bit of v ^ s that v has
    # set, else sets the lowest one it lacks
    d = 12
    g = _hypercube(d)
    ws = Workspace(Graph(g.offsets, g.cols), **({} if small_edges is None else {"small_edges": small_edges}))
    v = np.arange(1 << d)
    for s in (0, 0b101101110010, (1 << d) - 1):
        lv, par = run_single(ws, s)
        diff = v ^ s
        np.testing.assert_array_equal(lv, [bin(x).count("1") for x in diff])
        down = diff & v
        want = np.where(down > 0, v ^ (1 << (np.floor(np.log2(np.maximum(down, 1))).astype(np.int64))),
                        np.where(diff > 0, v | (diff & -diff), s))
        np.testing.assert_array_equal(par, want)


def _hubs_and_leaves(hubs, leaves, max_extra, seed):
    # vertex 0 -> hubs 1..hubs -> leaves; each leaf also links to up to max_extra other leaves, so
    # the level of leaves has sub-tiles of 2048 edges with anywhere from ~50 to 2049 entries
    rng = np.random.default_rng(seed)
    n = 1 + hubs + leaves
    edges = [(0, h) for h in range(1, hubs + 1)]
    edges += [(1 + (i % hubs), 1 + hubs + i) for i in range(leaves)]
    if max_extra:
        deg = rng.integers(0, max_extra + 1, size=leaves)
        for i in range(leaves):
            for j in rng.integers(0, leaves, size=int(deg[i])):
                if j != i:
                    edges.append((1 + hubs + i, 1 + hubs + int(j)))
    return gg.from_edges(n, edges)


@pytest.mark.parametrize("max_extra", [0, 1, 3, 40])
@pytest.mark.parametrize("mode", [BFS_MODE_AUTO, BFS_MODE_INSENSITIVE])
def test_frontiers_of_short_rows(max_extra, mode):
    g = _hubs_and_leaves(3, 9000, max_extra, seed=5 + max_extra)
    ws = Workspace(Graph(g.offsets, g.cols), mode=mode, small_edges=0)
    for s in (0, 1, g.n - 1):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [s])


def test_isolated_source_and_tiny_graphs():
    g = gg.from_edges(6, [(0, 1), (1, 2)])
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G)
    for s in range(6):
        lv, par = run_single(ws, s)
        assert_same(lv, par, g, [s])
    one = gg.from_edges(1, [])
    ws1 = Workspace(Graph(one.offsets, one.cols))
    lv, par = run_single(ws1, 0)
    assert lv.tolist() == [0] and par.tolist() == [0]


def test_hub_spanning_many_shares():
    # a star with 100k leaves: one vertex's row spans ~50 shares
    n = 100_001
    g = gg.from_edges(n, [(0, i) for i in range(1, n)] + [(5, 6), (7, 8)])
    G = Graph(g.offsets, g.cols)
    for mode in (BFS_MODE_AUTO, BFS_MODE_LEVEL):
        ws = Workspace(G, mode=mode)
        for s in (0, 17):
            lv, par = run_single(ws, s)
            assert_same(lv, par, g, [s])


def test_multiroot_disjoint_union():
    parts = [gg.grid(30, 20), gg.rmat(9, seed=3), gg.powerlaw_forest(2000, seed=1), gg.from_edges(3, [])]
    u, base = gg.disjoint_union(parts)
    roots = [int(base[0]) + 5, int(base[1]) + int(gg.pick_sources(parts[1], 1)[0]), int(base[2]), int(base[3]) + 1]
    G = Graph(u.offsets, u.cols)
    ws = Workspace(G)
    lv, par = ws.run_multiroot(roots)
    ws.sync()
    assert_same(lv.cpu().numpy(), par.cpu().numpy(), u, roots)
    # repeated and same-component roots
    roots2 = roots + [roots[0], int(base[0]) + 100]
    lv, par = ws.run_multiroot(roots2)
    ws.sync()
    assert_same(lv.cpu().numpy(), par.cpu().numpy(), u, roots2)


def test_level_stats_match_oracle(rmat14):
    g, G = rmat14
    for mode in (BFS_MODE_AUTO, BFS_MODE_LEVEL, BFS_MODE_INSENSITIVE):
        ws = Workspace(G, mode=mode)
        s = int(gg.pick_sources(g, 1, seed=33)[0])
        run_single(ws, s)
        n_l, e_l = ws.level_stats()
        lv = oracle.bfs_levels(g.offsets, g.cols, s)
        wn, we = oracle.level_stats(g.offsets, lv)
        assert n_l.tolist() == wn.tolist()
        assert e_l.tolist() == we.tolist()
        st = ws.stats()
        assert st["levels"] == len(wn) and st["reached"] == wn.sum() and st["edges"] == we.sum()


def test_determinism_repeated_runs(rmat14):
    g, G = rmat14
    ws = Workspace(G)
    s = int(gg.pick_sources(g, 1, seed=8)[0])
    first = run_single(ws, s)
    for _ in range(5):
        again = run_single(ws, s)
        assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1])


def test_certificate_without_parent_pass_inputs(rmat14):
    g, G = rmat14
    ws = Workspace(G)
    s = int(gg.pick_sources(g, 1, seed=77)[0])
    lv, par = run_single(ws, s)
    assert certify(g.offsets, g.cols, [s], lv, par) == []
    lv2, _ = run_single(ws, s, want_parent=False)
    assert np.array_equal(lv, lv2)


def test_errors(rmat14):
    g, G = rmat14
    ws = Workspace(G)
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(BFSError) as e:
        from paper_2209_08764_amd import bfs_run
        bfs_run(ws.handle, g.n, lv)
    assert e.value.status == _lib.BFS_ERANGE
    with pytest.raises(BFSError) as e:
        ws.set(BFS_OPT_MODE, 99)
    assert e.value.status == _lib.BFS_EINVAL
    bad = gg.Graph(np.array([0, 1, 1], np.int32), np.array([1], np.int32))
    with pytest.raises(BFSError) as e:
        Graph(bad.offsets, bad.cols, validate=True)
    assert e.value.status == _lib.BFS_EBADCSR


def test_small_stretches_handing_over_to_the_full_grid():
    # Low-degree sources on a larger R-MAT: the group runs one or two small
    # levels and hands a large frontier back to the whole grid (the hand-over
    # must not disturb workgroups still reading the entry level), from LDS or,
    # past 4096 entries, from its global entry arrays.
    g = gg.rmat(18, seed=41)
    G = Graph(g.offsets, g.cols)
    deg = g.degrees()
    cand = np.flatnonzero((deg > 0) & (deg <= 3))
    rng = np.random.default_rng(5)
    srcs = rng.choice(cand, 12, replace=False)
    for small in (16384, 2048, 0):
        ws = Workspace(G, small_edges=small)
        for s in srcs:
            lv, par = run_single(ws, s)
            assert_same(lv, par, g, [s])
        assert ws.stats()["status"] == 0


@pytest.mark.parametrize("push_edges", [0, 64, 1 << 20, 1 << 30])
@pytest.mark.parametrize("small_edges", [0, 16384])
def test_parent_rules_agree(push_edges, small_edges):
    # pushed (atomic minimum per edge) and pulled (first level-l entry of a
    # sorted row) parents must agree; the hub's parent is the last entry of
    # its 5000-long row, so the pull falls back to the whole-workgroup scan
    n = 5002
    edges = [(0, i) for i in range(1, 5001)] + [(5001, 5000)] + [(i, i + 1) for i in range(1, 60)]
    star = gg.from_edges(n, edges)
    g14 = gg.rmat(14, seed=23)
    for g, srcs in [(star, [5001, 0, 30]), (g14, list(gg.pick_sources(g14, 3, seed=4)))]:
        G = Graph(g.offsets, g.cols)
        ws = Workspace(G, small_edges=small_edges, push_edges=push_edges)
        for s in srcs:
            lv, par = run_single(ws, s)
            assert_same(lv, par, g, [s])


def test_default_grid_follows_graph_size():
    # one workgroup per 16384 edges, a multiple of 8, at least 64; an explicit grid wins
    g = gg.rmat(12, seed=33)
    G = Graph(g.offsets, g.cols)
    s = int(gg.pick_sources(g, 1, seed=2)[0])
    ws = Workspace(G)
    lv, par = run_single(ws, s)
    assert_same(lv, par, g, [s])
    assert ws.stats()["grid"] == 64
    ws = Workspace(G, grid=40)
    lv, par = run_single(ws, s)
    assert_same(lv, par, g, [s])
    assert ws.stats()["grid"] == 40
    big = gg.rmat(17, seed=34)
    ws = Workspace(Graph(big.offsets, big.cols))
    run_single(ws, int(gg.pick_sources(big, 1, seed=3)[0]))
    want = max(64, (big.m // 16384 + 7) // 8 * 8)
    assert 64 < want < 512 and ws.stats()["grid"] == want  # below what two workgroups per CU allow


@pytest.mark.parametrize("group", [1, 2, 5, 16, 64])
def test_group_sizes_do_not_change_results(group):
    # small levels run on `group` workgroups (capped at the grid): high-diameter graphs whose
    # levels stay small throughout, and R-MAT levels that enter and leave the group
    cases = [(gg.grid(64, 64), [0, 2080]), (gg.grid(1, 3000), [0, 1500]), (gg.grid(200, 90), [0, 9000]),
             (gg.powerlaw_forest(1 << 13, seed=3), None), (gg.rmat(14, seed=21), None)]
    for g, srcs in cases:
        G = Graph(g.offsets, g.cols)
        for small in (16384, 1 << 30, 3000):
            ws = Workspace(G, group=group, small_edges=small)
            for s in (srcs if srcs is not None else gg.pick_sources(g, 2, seed=group)):
                lv, par = run_single(ws, s)
                assert_same(lv, par, g, [s])
                assert ws.stats()["status"] == 0
            lv, _ = run_single(ws, int(srcs[0]) if srcs is not None else 0, want_parent=False)
            assert np.array_equal(lv, oracle.bfs(g.offsets, g.cols, int(srcs[0]) if srcs is not None else 0)[0])


def test_a_wait_that_times_out_is_reported_and_the_next_run_is_clean():
    # a 1-tick limit on the persistent loop's waits makes the first wait that is not over
    # within its first 32 polls record a device failure; every workgroup leaves at its next
    # wait, the run reports BFS_EDEVICE, and the next run (default limit) is bit-exact
    from paper_2209_08764_amd import BFSError, _lib
    g = gg.rmat(20, seed=73)
    ws = Workspace(Graph(g.offsets, g.cols))
    s = int(gg.pick_sources(g, 1, seed=74)[0])
    lib = _lib.load()
    _lib.check(lib.bfs_workspace_set_spin_ticks(ws.handle, 1), "bfs_workspace_set_spin_ticks")
    ws.run(s)
    with pytest.raises(BFSError) as err:
        ws.sync()
    assert err.value.status == _lib.BFS_EDEVICE
    assert ws.stats()["status"] == _lib.BFS_EDEVICE
    _lib.check(lib.bfs_workspace_set_spin_ticks(ws.handle, 0), "bfs_workspace_set_spin_ticks")
    lv, par = run_single(ws, s)
    assert_same(lv, par, g, [s])
    assert ws.stats()["status"] == 0


def test_run_status_reads_the_device_status_without_a_wait():
    from paper_2209_08764_amd import BFSError, _lib
    g = gg.rmat(20, seed=75)
    G = Graph(g.offsets, g.cols)
    s = int(gg.pick_sources(g, 1, seed=76)[0])
    plain = Workspace(G)
    plain.run(s)
    torch.cuda.synchronize()
    with pytest.raises(BFSError) as err:        # the option was not set for that run
        plain.run_status()
    assert err.value.status == _lib.BFS_EINVAL
    ws = Workspace(G, host_status=1)
    ws.run(s)
    torch.cuda.synchronize()
    assert ws.run_status() == _lib.BFS_OK
    _lib.check(_lib.load().bfs_workspace_set_spin_ticks(ws.handle, 1), "bfs_workspace_set_spin_ticks")
    ws.run(s)
    torch.cuda.synchronize()
    assert ws.run_status() == _lib.BFS_EDEVICE
    _lib.check(_lib.load().bfs_workspace_set_spin_ticks(ws.handle, 0), "bfs_workspace_set_spin_ticks")
    lv, par = run_single(ws, s)
    assert ws.run_status() == _lib.BFS_OK
    assert_same(lv, par, g, [s])
