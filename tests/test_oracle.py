"""Pins for the CPU oracle (no GPU): brute force, closed forms, invariants.

Each test checks the oracle against something other than itself: the
Floyd-Warshall distance matrix (a different algorithm), closed-form answers
on structured graphs, scipy's shortest paths and the invariant certificate.
The mutant tests show that the pins have teeth: plausible mistakes in a BFS
(a wrong parent rule, a dropped +1, a stale visited check) fail them.
"""
import itertools
import math
import random

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import brute
from oracle.certify import certify


def _graph_from_mask(n, mask):
    pairs = list(itertools.combinations(range(n), 2))
    edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
    return gg.from_edges(n, edges)


def _check_vs_brute(g, roots):
    A = brute.adjacency(g.n, g.offsets, g.cols)
    D = brute.floyd_warshall(A)
    lv, par = oracle.bfs(g.offsets, g.cols, roots)
    blv, bpar = brute.level_parent_from_distances(A, D, roots)
    np.testing.assert_array_equal(lv, blv)
    np.testing.assert_array_equal(par, bpar)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_small_graphs_vs_floyd_warshall(n):
    npairs = n * (n - 1) // 2
    for mask in range(1 << npairs):
        g = _graph_from_mask(n, mask)
        A = brute.adjacency(n, g.offsets, g.cols)
        D = brute.floyd_warshall(A)
        for s in range(n):
            lv, par = oracle.bfs(g.offsets, g.cols, s)
            blv, bpar = brute.level_parent_from_distances(A, D, [s])
            assert np.array_equal(lv, blv), (n, mask, s)
            assert np.array_equal(par, bpar), (n, mask, s)


def test_n6_graphs_vs_floyd_warshall():
    # every 16th of the 32768 labelled graphs on 6 vertices, all sources
    n = 6
    for mask in range(0, 1 << 15, 16):
        g = _graph_from_mask(n, mask)
        A = brute.adjacency(n, g.offsets, g.cols)
        D = brute.floyd_warshall(A)
        for s in range(n):
            lv, par = oracle.bfs(g.offsets, g.cols, s)
            blv, bpar = brute.level_parent_from_distances(A, D, [s])
            assert np.array_equal(lv, blv) and np.array_equal(par, bpar), (mask, s)


@pytest.mark.parametrize("seed", range(12))
def test_random_graphs_up_to_64_vs_floyd_warshall(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 64)
    p = rng.choice([0.02, 0.05, 0.1, 0.2, 0.5])
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    g = gg.from_edges(n, edges)
    for s in rng.sample(range(n), min(n, 6)):
        _check_vs_brute(g, [s])
    # several roots: distance to the nearest root
    _check_vs_brute(g, rng.sample(range(n), min(n, 3)))


def test_grid_closed_form():
    W, H = 37, 23
    g = gg.grid(W, H)
    for (r0, c0) in [(0, 0), (11, 17), (H - 1, W - 1), (0, W - 1)]:
        s = r0 * W + c0
        lv, par = oracle.bfs(g.offsets, g.cols, s)
        r, c = np.divmod(np.arange(W * H), W)
        np.testing.assert_array_equal(lv, np.abs(r - r0) + np.abs(c - c0))
        # neighbour ids ascend as up < left < right < down
        want = np.where(r > r0, (r - 1) * W + c,
                        np.where(c > c0, r * W + c - 1,
                                 np.where(c < c0, r * W + c + 1,
                                          np.where(r < r0, (r + 1) * W + c, s))))
        np.testing.assert_array_equal(par, want)


def test_path_cycle_star_complete():
    n = 41
    path = gg.from_edges(n, [(i, i + 1) for i in range(n - 1)])
    for s in (0, 7, n - 1):
        lv, par = oracle.bfs(path.offsets, path.cols, s)
        i = np.arange(n)
        np.testing.assert_array_equal(lv, np.abs(i - s))
        np.testing.assert_array_equal(par, np.where(i > s, i - 1, np.where(i < s, i + 1, s)))
    # even cycle: the antipode has two neighbours one level up, takes the smaller id
    L = 20
    cyc = gg.from_edges(L, [(i, (i + 1) % L) for i in range(L)])
    lv, par = oracle.bfs(cyc.offsets, cyc.cols, 0)
    i = np.arange(L)
    np.testing.assert_array_equal(lv, np.minimum(i, L - i))
    assert par[L // 2] == L // 2 - 1
    # odd cycle
    L = 21
    cyc = gg.from_edges(L, [(i, (i + 1) % L) for i in range(L)])
    lv, _ = oracle.bfs(cyc.offsets, cyc.cols, 3)
    i = np.arange(L)
    np.testing.assert_array_equal(lv, np.minimum((i - 3) % L, (3 - i) % L))
    # star from the centre and from a leaf
    star = gg.from_edges(10, [(0, i) for i in range(1, 10)])
    lv, par = oracle.bfs(star.offsets, star.cols, 0)
    assert lv[0] == 0 and (lv[1:] == 1).all() and (par[1:] == 0).all()
    lv, par = oracle.bfs(star.offsets, star.cols, 5)
    assert lv[5] == 0 and lv[0] == 1 and par[0] == 5
    assert all(lv[i] == 2 and par[i] == 0 for i in range(1, 10) if i != 5)
    # K_n: every other vertex at level 1 with parent s
    K = gg.from_edges(12, list(itertools.combinations(range(12), 2)))
    lv, par = oracle.bfs(K.offsets, K.cols, 4)
    assert (lv == np.where(np.arange(12) == 4, 0, 1)).all() and (par == 4).all()


def test_complete_bipartite_and_heap_tree():
    a, b = 5, 7
    kb = gg.from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])
    lv, par = oracle.bfs(kb.offsets, kb.cols, 2)
    i = np.arange(a + b)
    np.testing.assert_array_equal(lv, np.where(i == 2, 0, np.where(i < a, 2, 1)))
    np.testing.assert_array_equal(par[a:], 2)                 # right side hangs off the source
    np.testing.assert_array_equal(par[[0, 1, 3, 4]], a)        # left side: smallest right vertex
    n = 200
    heap = gg.from_edges(n, [(v, (v - 1) // 2) for v in range(1, n)])
    lv, par = oracle.bfs(heap.offsets, heap.cols, 0)
    v = np.arange(n)
    np.testing.assert_array_equal(lv, np.floor(np.log2(v + 1)).astype(np.int32))
    np.testing.assert_array_equal(par[1:], (v[1:] - 1) // 2)


def _gen_petersen(n, k):
    # generalised Petersen graph GP(n, k): outer cycle 0..n-1, spokes i - n+i, inner i+n - (i+k mod n)+n
    return gg.from_edges(2 * n, [(i, (i + 1) % n) for i in range(n)] + [(i, n + i) for i in range(n)]
                         + [(n + i, n + (i + k) % n) for i in range(n)])


def test_distance_regular_level_counts():
    # distance-regular graphs have the same number of vertices at distance i from every vertex:
    # Petersen GP(5,2) 1,3,6; dodecahedron GP(10,2) 1,3,6,6,3,1; Desargues GP(10,3) 1,3,6,6,3,1;
    # hypercube Q_d the binomial coefficients C(d, i).  Petersen and the dodecahedron have odd
    # cycles (girth 5); Desargues and Q_d are bipartite.
    cases = [(_gen_petersen(5, 2), [1, 3, 6]), (_gen_petersen(10, 2), [1, 3, 6, 6, 3, 1]),
             (_gen_petersen(10, 3), [1, 3, 6, 6, 3, 1])]
    for d in (3, 5, 7):
        q = gg.from_edges(1 << d, [(v, v ^ (1 << b)) for v in range(1 << d) for b in range(d) if v < v ^ (1 << b)])
        cases.append((q, [math.comb(d, i) for i in range(d + 1)]))
    for g, counts in cases:
        for s in range(g.n):
            lv, _ = oracle.bfs(g.offsets, g.cols, s)
            assert np.bincount(lv).tolist() == counts, (g.n, s)


def test_petersen_parents_by_hand():
    # GP(5,2) from vertex 0: level 1 = {1, 4, 5}; every level-2 vertex has exactly one neighbour
    # at level 1 (girth 5), so its parent is that neighbour: 2-1, 3-4, 6-1, 7-5, 8-5, 9-4
    g = _gen_petersen(5, 2)
    lv, par = oracle.bfs(g.offsets, g.cols, 0)
    assert lv.tolist() == [0, 1, 2, 2, 1, 1, 2, 2, 2, 2]
    assert par.tolist() == [0, 0, 1, 4, 0, 0, 1, 5, 5, 4]


def test_hypercube_parents_closed_form():
    # Q_d from s: level(v) = popcount(v ^ s); the closer neighbours flip one bit of v ^ s, and the
    # smallest of them clears the highest such bit that v has set, else sets the lowest one v lacks
    d, s = 8, 0b10110010
    q = gg.from_edges(1 << d, [(v, v ^ (1 << b)) for v in range(1 << d) for b in range(d) if v < v ^ (1 << b)])
    lv, par = oracle.bfs(q.offsets, q.cols, s)
    for v in range(1 << d):
        diff = v ^ s
        assert lv[v] == bin(diff).count("1")
        down = diff & v
        want = v ^ (1 << (down.bit_length() - 1)) if down else (v | (diff & -diff) if diff else s)
        assert par[v] == want, v


def test_empty_and_isolated():
    g = gg.from_edges(5, [])
    lv, par = oracle.bfs(g.offsets, g.cols, 3)
    np.testing.assert_array_equal(lv, [-1, -1, -1, 0, -1])
    np.testing.assert_array_equal(par, [-1, -1, -1, 3, -1])
    g = gg.from_edges(6, [(0, 1), (1, 2)])
    lv, par = oracle.bfs(g.offsets, g.cols, 5)
    assert lv.tolist() == [-1] * 5 + [0] and par.tolist() == [-1] * 5 + [5]
    with pytest.raises(ValueError):
        oracle.bfs(g.offsets, g.cols, 6)


@pytest.mark.parametrize("make", [lambda: gg.rmat(12, seed=3), lambda: gg.grid(64, 50),
                                  lambda: gg.powerlaw_forest(5000, seed=2),
                                  lambda: gg.erdos_renyi(4000, 3.0, seed=5)])
def test_certificate_and_scipy_on_generated_graphs(make):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path

    g = make()
    srcs = gg.pick_sources(g, 3, seed=11)
    A = sp.csr_matrix((np.ones(g.m), g.cols, g.offsets), shape=(g.n, g.n))
    for s in srcs:
        lv, par = oracle.bfs(g.offsets, g.cols, s)
        assert certify(g.offsets, g.cols, [s], lv, par) == []
        d = shortest_path(A, unweighted=True, indices=[int(s)])[0]
        np.testing.assert_array_equal(lv, np.where(np.isinf(d), -1, d).astype(np.int32))


# ---- mutants: the pins must reject plausible mistakes --------------------------------

def _mutant_first_discoverer_parent(g, s):
    n = g.n
    lv = np.full(n, -1)
    par = np.full(n, -1)
    lv[s], par[s] = 0, s
    q = [s]
    for u in q:
        for v in g.cols[g.offsets[u]:g.offsets[u + 1]]:
            if lv[v] == -1:
                lv[v], par[v] = lv[u] + 1, u
                q.append(v)
    return lv, par


def _mutant_lifo(g, s):
    # a stack instead of a queue: levels are no longer distances
    n = g.n
    lv = np.full(n, -1)
    lv[s] = 0
    st = [s]
    while st:
        u = st.pop()
        for v in g.cols[g.offsets[u]:g.offsets[u + 1]]:
            if lv[v] == -1:
                lv[v] = lv[u] + 1
                st.append(v)
    return lv, oracle.parents(g.offsets, g.cols, lv)


def _mutant_skip_last_neighbour(g, s):
    n = g.n
    lv = np.full(n, -1)
    lv[s] = 0
    q = [s]
    for u in q:
        for v in g.cols[g.offsets[u]:max(g.offsets[u + 1] - 1, g.offsets[u])]:
            if lv[v] == -1:
                lv[v] = lv[u] + 1
                q.append(v)
    return lv, oracle.parents(g.offsets, g.cols, lv)


@pytest.mark.parametrize("mutant", [_mutant_first_discoverer_parent, _mutant_lifo, _mutant_skip_last_neighbour])
def test_pins_reject_mutants(mutant):
    g = gg.rmat(10, seed=9)
    s = int(gg.pick_sources(g, 1, seed=4)[0])
    lv, par = mutant(g, s)
    assert certify(g.offsets, g.cols, [s], lv, par) != []
    small = gg.from_edges(8, [(0, 5), (0, 6), (5, 2), (6, 1), (2, 7), (1, 7), (3, 4), (4, 0), (3, 6)])
    A = brute.adjacency(8, small.offsets, small.cols)
    D = brute.floyd_warshall(A)
    bad = 0
    for s in range(8):
        lv, par = mutant(small, s)
        blv, bpar = brute.level_parent_from_distances(A, D, [s])
        bad += not (np.array_equal(lv, blv) and np.array_equal(par, bpar))
    assert bad > 0


def test_certificate_rejects_planted_errors():
    g = gg.rmat(11, seed=2)
    s = int(gg.pick_sources(g, 1, seed=1)[0])
    lv, par = oracle.bfs(g.offsets, g.cols, s)
    assert certify(g.offsets, g.cols, [s], lv, par) == []
    reached = np.flatnonzero(lv > 1)
    v = int(reached[len(reached) // 2])
    bad_lv = lv.copy(); bad_lv[v] += 1
    assert certify(g.offsets, g.cols, [s], bad_lv, par) != []
    bad_par = par.copy()
    nb = g.cols[g.offsets[v]:g.offsets[v + 1]]
    others = [u for u in nb if lv[u] == lv[v] - 1 and u != par[v]]
    bad_par[v] = others[0] if others else s
    assert certify(g.offsets, g.cols, [s], lv, bad_par) != []
    unreached = np.flatnonzero(lv == -1)
    if unreached.size:
        bad_lv = lv.copy(); bad_lv[unreached[0]] = 3
        assert certify(g.offsets, g.cols, [s], bad_lv, par) != []


# ---- batched oracle ---------------------------------------------------------------------

def test_batch_u8_matches_single_source_and_overflow():
    g = gg.rmat(11, seed=5)
    srcs = gg.pick_sources(g, 9, seed=2)
    out, ovf = oracle.bfs_batch_u8(g.offsets, g.cols, srcs)
    assert not ovf and out.shape == (g.n, 9)
    for j, s in enumerate(srcs):
        lv = oracle.bfs_levels(g.offsets, g.cols, s)
        np.testing.assert_array_equal(out[:, j], np.where(lv < 0, 255, lv).astype(np.uint8))
    path = gg.from_edges(300, [(i, i + 1) for i in range(299)])
    out, ovf = oracle.bfs_batch_u8(path.offsets, path.cols, [0, 150])
    assert ovf and out[254, 0] == 254 and out[255, 0] == 255 and out[299, 1] == 149


def test_level_stats_sums():
    g = gg.rmat(12, seed=1)
    s = int(gg.pick_sources(g, 1)[0])
    lv = oracle.bfs_levels(g.offsets, g.cols, s)
    n_l, e_l = oracle.level_stats(g.offsets, lv)
    deg = g.degrees()
    assert n_l.sum() == (lv >= 0).sum()
    assert e_l.sum() == deg[lv >= 0].sum()
    assert n_l[0] == 1 and e_l[0] == deg[s]
