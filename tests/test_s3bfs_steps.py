"""Pins for the primitive-by-primitive step model (oracle/s3bfs_steps.py), no GPU.

The chunk starts (the scatter form of the paper's Find-StartExpPoint) are
checked against a binary search done by numpy's searchsorted; the ownership
filter and the concatenation against their set semantics; the whole round
loop against the plain BFS oracle (itself pinned by brute force), with and
without the modelled race between workers.
"""
import random

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import s3bfs_steps as st


def _split_by_search(incl, e_l, S):
    incl = np.asarray(incl, dtype=np.int64)
    out = []
    for t in range(-(-e_l // S) if S else 0):
        g = t * S
        j = int(np.searchsorted(incl, g, side="right"))
        a = int(incl[j - 1]) if j > 0 else 0
        out.append((j, g - a))
    return out


@pytest.mark.parametrize("seed", range(40))
def test_find_start_exp_point_equals_binary_search(seed):
    rng = random.Random(seed)
    n_l = rng.choice([1, 2, 3, 7, 64, 65, 300])
    degs = [rng.choice([0, 0, 1, 2, 3, 5, 17, 100, 2049]) for _ in range(n_l)]
    incl = st.running_totals(degs)
    e_l = incl[-1]
    for P_l in {1, 2, 3, 7, 64, max(e_l, 1), e_l + 5}:
        P_l = min(P_l, e_l) if e_l else 0
        if P_l == 0:
            assert st.chunk_starts(incl, e_l, P_l) == []
            continue
        S = st.chunk_size(e_l, P_l)
        got = st.chunk_starts(incl, e_l, P_l)
        want = _split_by_search(incl, e_l, S)
        assert got[:len(want)] == want
        assert all(x is None for x in got[len(want):])
        # every share start points at a vertex with an edge at that offset
        for (j, off) in want:
            assert 0 <= off < degs[j]


def test_find_start_exp_point_hub_and_tiny():
    incl = st.running_totals([1, 100000, 0, 2])
    got = st.chunk_starts(incl, incl[-1], 0, size=2048)
    assert got == []
    got = st.chunk_starts(incl, incl[-1], 49, size=2048)
    assert got[0] == (0, 0) and got[1] == (1, 2047) and got[48] == (1, 48 * 2048 - 1)
    # fewer edges than chunks asked for
    incl = st.running_totals([2, 1])
    got = st.chunk_starts(incl, 3, 3)
    assert got == [(0, 0), (0, 1), (1, 0)]


def test_running_totals_and_row_lengths():
    g = gg.grid(5, 4)
    deg = st.row_lengths([0, 7, 19], g.offsets)
    assert deg == [2, 4, 2]        # a corner, an inner vertex, the far corner
    assert st.running_totals(deg) == [2, 6, 8]
    assert st.running_totals([]) == []


@pytest.mark.parametrize("P", [1, 2, 5, 64, 10 ** 6])
@pytest.mark.parametrize("race", [None, 1, 2])
def test_parallel_bfs_equals_plain_definition(P, race):
    g = gg.rmat(9, seed=7)
    for s in gg.pick_sources(g, 3, seed=P + (race or 0)):
        d, stats = st.level_synchronous_bfs(g.offsets, g.cols, int(s), P, race=race)
        lv = oracle.bfs_levels(g.offsets, g.cols, s)
        np.testing.assert_array_equal(np.array(d), lv)
        n_l, e_l = oracle.level_stats(g.offsets, lv)
        assert [x[0] for x in stats] == n_l.tolist()
        assert [x[1] for x in stats] == e_l.tolist()


@pytest.mark.parametrize("S", [1, 3, 64, 2048])
def test_parallel_bfs_fixed_grain(S):
    g = gg.grid(20, 9)
    d, stats = st.level_synchronous_bfs(g.offsets, g.cols, 0, 10 ** 9, race=5, size=S)
    lv = oracle.bfs_levels(g.offsets, g.cols, 0)
    np.testing.assert_array_equal(np.array(d), lv)


def test_dedup_keeps_exactly_one_copy():
    # a vertex listed by several workers survives once, in the list of its final claimant
    claim = {7: 2, 8: 0}
    lists = [[7, 8], [7], [7]]
    kept, sizes = st.keep_claimed(lists, claim)
    assert kept == [[8], [], [7]] and sizes == [1, 0, 1]
    assert st.concatenate(kept, st.running_totals(sizes)) == [8, 7]


@pytest.mark.parametrize("seed", range(20))
def test_filter_and_concatenate_are_set_exact(seed):
    # random lists (a vertex in several lists, at most once in each, as a worker lists its own
    # claims once) and a random final claimant per vertex: the output holds every claimed vertex
    # exactly once, and each list's survivors keep their order in one block
    rng = random.Random(seed)
    workers = rng.randint(1, 9)
    lists = [rng.sample(range(30), rng.randint(0, 12)) for _ in range(workers)]
    claim = {}
    for v in {x for lst in lists for x in lst}:
        holders = [w for w, lst in enumerate(lists) if v in lst]
        claim[v] = rng.choice(holders)
    kept, sizes = st.keep_claimed(lists, claim)
    out = st.concatenate(kept, st.running_totals(sizes))
    assert sorted(out) == sorted(claim)
    pos = 0
    for w in range(workers):
        assert out[pos:pos + sizes[w]] == [v for v in lists[w] if claim[v] == w]
        pos += sizes[w]
