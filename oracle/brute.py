"""Brute-force all-pairs distances (test infrastructure only).

Floyd-Warshall with unit weights on graphs of at most a few dozen vertices.
It is a different algorithm from the FIFO search in oracle.c (dynamic
programming over intermediate vertices, no queue), so agreement between the
two pins the oracle's level output; the parent then follows from the
definition (smallest-id neighbour one hop closer) applied to the distance
matrix.
"""
from __future__ import annotations

import numpy as np


def adjacency(n: int, offsets, cols) -> np.ndarray:
    A = np.zeros((n, n), dtype=bool)
    for v in range(n):
        for e in range(int(offsets[v]), int(offsets[v + 1])):
            A[v, int(cols[e])] = True
    return A


def floyd_warshall(A: np.ndarray) -> np.ndarray:
    """All-pairs hop distances; -1 where unreachable."""
    n = A.shape[0]
    INF = n + 1
    D = np.where(A, 1, INF).astype(np.int64)
    np.fill_diagonal(D, 0)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    D[D >= INF] = -1
    return D


def level_parent_from_distances(A: np.ndarray, D: np.ndarray, roots):
    """level/parent for a root set: distance to the nearest root, min-id parent."""
    n = A.shape[0]
    roots = list(np.atleast_1d(roots))
    level = np.full(n, -1, np.int64)
    for v in range(n):
        ds = [D[r, v] for r in roots if D[r, v] >= 0]
        if ds:
            level[v] = min(ds)
    parent = np.full(n, -1, np.int64)
    for v in range(n):
        if level[v] == 0:
            parent[v] = v
        elif level[v] > 0:
            cands = [u for u in range(n) if A[v, u] and level[u] == level[v] - 1]
            parent[v] = min(cands)
    return level.astype(np.int32), parent.astype(np.int32)
