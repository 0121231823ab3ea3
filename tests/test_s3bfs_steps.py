"""Pins for the paper's step-by-step reference (oracle/s3bfs_steps.py), no GPU.

The split reference (the paper's Find-StartExpPoint scatter) is checked
against a binary search done by numpy's searchsorted; the whole Figure 1
loop is checked against the plain BFS oracle (itself pinned by brute force),
with and without the modelled benign race.
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
    incl = st.inclusive_prefix_sum(degs)
    e_l = incl[-1]
    for P_l in {1, 2, 3, 7, 64, max(e_l, 1), e_l + 5}:
        P_l = min(P_l, e_l) if e_l else 0
        if P_l == 0:
            assert st.find_start_exp_point(incl, e_l, P_l) == []
            continue
        S = st.share_size(e_l, P_l)
        got = st.find_start_exp_point(incl, e_l, P_l)
        want = _split_by_search(incl, e_l, S)
        assert got[:len(want)] == want
        assert all(x is None for x in got[len(want):])
        # every share start points at a vertex with an edge at that offset
        for (j, off) in want:
            assert 0 <= off < degs[j]


def test_find_start_exp_point_hub_and_tiny():
    incl = st.inclusive_prefix_sum([1, 100000, 0, 2])
    got = st.find_start_exp_point(incl, incl[-1], 0, S=2048)
    assert got == []
    got = st.find_start_exp_point(incl, incl[-1], 49, S=2048)
    assert got[0] == (0, 0) and got[1] == (1, 2047) and got[48] == (1, 48 * 2048 - 1)
    # e_l smaller than the number of shares asked for
    incl = st.inclusive_prefix_sum([2, 1])
    got = st.find_start_exp_point(incl, 3, 3)
    assert got == [(0, 0), (0, 1), (1, 0)]


@pytest.mark.parametrize("P", [1, 2, 5, 64, 10 ** 6])
@pytest.mark.parametrize("race", [None, 1, 2])
def test_parallel_bfs_equals_plain_definition(P, race):
    g = gg.rmat(9, seed=7)
    for s in gg.pick_sources(g, 3, seed=P + (race or 0)):
        d, stats = st.parallel_bfs(g.offsets, g.cols, int(s), P, race=race)
        lv = oracle.bfs_levels(g.offsets, g.cols, s)
        got = np.array([-1 if x is None else x for x in d])
        np.testing.assert_array_equal(got, lv)
        n_l, e_l = oracle.level_stats(g.offsets, lv)
        assert [x[0] for x in stats] == n_l.tolist()
        assert [x[1] for x in stats] == e_l.tolist()


@pytest.mark.parametrize("S", [1, 3, 64, 2048])
def test_parallel_bfs_fixed_grain(S):
    g = gg.grid(20, 9)
    d, stats = st.parallel_bfs(g.offsets, g.cols, 0, 10 ** 9, race=5, S=S)
    lv = oracle.bfs_levels(g.offsets, g.cols, 0)
    np.testing.assert_array_equal(np.array(d), lv)


def test_dedup_keeps_exactly_one_copy():
    # a vertex claimed by several threads survives once
    owner = {7: 2, 8: 0}
    Q = [[7, 8], [7], [7]]
    Qn, sizes = st.deduplicate(Q, owner)
    assert Qn == [[8], [], [7]] and sizes == [1, 0, 1]
    assert st.linearize(Qn, st.inclusive_prefix_sum(sizes)) == [8, 7]
