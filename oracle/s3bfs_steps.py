"""The paper's S3BFS steps written out in plain Python (test infrastructure only).

This follows Figure 1 (Parallel-BFS(s, P)) and the Algorithm and Analysis
paragraphs in the paper's order and notation, with the P_l "threads" of each
step simulated one after another.  It is slow and meant for small graphs.
It is the reference for the GPU library's primitives (degree gather, prefix
sum, the start point of each share) and for its per-level statistics
(n_l, e_l), and it shows that the owner-based de-duplication returns the same
levels as the plain definition even under the paper's benign race.

Readings where the figure is silent or garbled (each is also listed in the
design notes):
  * EXPLORE-VERTEX has no body in Figure 1; from the Algorithm paragraph:
    each thread scans its share of the level's edges and, for each neighbour
    v with d[v] = infinity, sets d[v] = l, Owner[v] = its id and appends v
    to its private queue.
  * Share rule: S = ceil(e_l / P_l); share t covers global edge positions
    [t*S, min((t+1)*S, e_l)).
  * Find-StartExpPoint: the EdgeSum entry j covering [a, b) is the start of
    every share t with ceil(a/S) <= t <= ceil(b/S) - 1, at edge t*S - a of
    that vertex (a scatter instead of a binary search).
  * The copy loop of the linearisation runs over the half-open range
    [Offset, Offset + |Q[i]|).
"""
from __future__ import annotations

import random

INF = None


def degree_gather(cur_level_vertices, offsets):
    """EdgeSum[u] = Degree[CurLevelVertices[u]] (Figure 1, degree gather)."""
    return [int(offsets[v + 1]) - int(offsets[v]) for v in cur_level_vertices]


def inclusive_prefix_sum(x):
    """Parallel-Prefix-Sum of Figure 1, written sequentially (inclusive)."""
    out, acc = [], 0
    for a in x:
        acc += int(a)
        out.append(acc)
    return out


def share_size(e_l: int, P_l: int) -> int:
    return -(-e_l // P_l) if P_l > 0 else 0


def find_start_exp_point(edge_sum, e_l: int, P_l: int, S: int | None = None):
    """Start (vertex index, edge within that vertex) of each of the P_l shares.

    edge_sum is the inclusive prefix sum of the frontier degrees.  Returns a
    list of length P_l whose entry t is (j, offset) or None for an empty share.
    A given share size S overrides ceil(e_l / P_l).
    """
    S = share_size(e_l, P_l) if S is None else S
    start = [None] * P_l
    if S <= 0:
        return start
    a = 0
    for j, b in enumerate(edge_sum):
        b = int(b)
        t_s = -(-a // S)          # first share that starts inside [a, b)
        t_e = -(-b // S) - 1      # last share that starts inside [a, b)
        for t in range(t_s, min(t_e, P_l - 1) + 1):
            start[t] = (j, t * S - a)
        a = b
    return start


def explore_vertex(cur, edge_sum, start, d, offsets, cols, e_l, P_l, l, owner, S=None, race=None):
    """EXPLORE-VERTEX: returns the private queues Q[0..P_l-1].

    race=None runs the shares one after another.  race=<seed> models the
    benign race: every thread reads d[] as it was at the start of the level
    (plus its own earlier writes, which program order makes visible to it),
    then the threads' writes land in a seeded random order (last writer wins
    on Owner).
    """
    S = share_size(e_l, P_l) if S is None else S
    Q = [[] for _ in range(P_l)]
    snapshot = list(d) if race is not None else None
    writes = []
    for t in range(P_l):
        if start[t] is None:
            continue
        j, off = start[t]
        g, g_end = t * S, min((t + 1) * S, e_l)
        mine = set()
        while g < g_end:
            u = cur[j]
            row0 = int(offsets[u])
            deg = int(offsets[u + 1]) - row0
            while off < deg and g < g_end:
                v = int(cols[row0 + off])
                if snapshot is None:
                    unvisited = d[v] is INF
                else:
                    unvisited = snapshot[v] is INF and v not in mine
                if unvisited:
                    if snapshot is None:
                        d[v] = l
                        owner[v] = t
                    else:
                        mine.add(v)
                        writes.append((t, v))
                    Q[t].append(v)
                off += 1
                g += 1
            j += 1
            off = 0
    if snapshot is not None:
        rng = random.Random(race)
        rng.shuffle(writes)
        for t, v in writes:
            d[v] = l
            owner[v] = t
    return Q


def deduplicate(Q, owner):
    """Keep v in Q[i] only if Owner[v] = i; returns (Q, Sizes)."""
    Qn = [[v for v in q if owner[v] == i] for i, q in enumerate(Q)]
    return Qn, [len(q) for q in Qn]


def linearize(Q, sizes_incl):
    """Copy the private queues into one array at the prefix-sum offsets."""
    total = sizes_incl[-1] if sizes_incl else 0
    out = [None] * total
    for i, q in enumerate(Q):
        offset = 0 if i == 0 else sizes_incl[i - 1]
        for j in range(offset, offset + len(q)):
            out[j] = q[j - offset]
    return out


def parallel_bfs(offsets, cols, s, P, race=None, S=None):
    """Figure 1.  Returns (d as a list with None for infinity, per-level stats).

    stats[k] = (n_l, e_l) of the k-th processed frontier (level k of the
    search), the work accounting of the Analysis paragraph.
    """
    n = len(offsets) - 1
    d = [INF] * n
    owner = [P] * n
    d[s] = 0
    owner[s] = 0
    cur = [s]
    l = 0
    stats = []
    while len(cur) > 0:
        n_l = len(cur)
        l += 1
        edge_sum = inclusive_prefix_sum(degree_gather(cur, offsets))
        e_l = edge_sum[n_l - 1]
        stats.append((n_l, e_l))
        # with a fixed share size (the GPU's grain) the share count follows it
        P_l = min(P, e_l) if S is None else share_size(e_l, S)
        if P_l == 0:
            break
        start = find_start_exp_point(edge_sum, e_l, P_l, S)
        Q = explore_vertex(cur, edge_sum, start, d, offsets, cols, e_l, P_l, l, owner, S, race)
        Q, sizes = deduplicate(Q, owner)
        cur = linearize(Q, inclusive_prefix_sum(sizes))
    return d, stats
