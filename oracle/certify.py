"""Exactness certificate for a (level, parent) pair (test infrastructure only).

For a symmetric graph and a root set R, the checks below hold for the exact
answer and for nothing else, so they pin a result at any size without
trusting any BFS implementation:

  I1  every root has level 0 and parent = itself; no other vertex has level 0
  I2  for every edge (u, v): u reached <=> v reached, and if both are reached
      |level[u] - level[v]| <= 1
  I3  every reached non-root v has parent[v] in N(v) with
      level[parent[v]] = level[v] - 1, and no smaller-id neighbour one level
      up; every unreached v has parent -1
  I4  the reached set is the union of the roots' connected components

I1 + I3 give a path of length level[v] from a root, so dist <= level; I2
along a shortest path gives level <= dist; I4 makes "unreached" exact.  So
level = distance and parent is the unique min-id choice.  Components are
taken from scipy's connected_components (a library routine).
"""
from __future__ import annotations

import numpy as np


def components(offsets, cols) -> np.ndarray:
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    n = len(offsets) - 1
    data = np.ones(len(cols), dtype=np.int8)
    A = sp.csr_matrix((data, np.asarray(cols, np.int64), np.asarray(offsets, np.int64)), shape=(n, n))
    _, lab = connected_components(A, directed=False)
    return lab


def certify(offsets, cols, roots, level, parent=None, comp_labels=None):
    """Return a list of violated invariants (empty when the result is exact)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    level = np.asarray(level, dtype=np.int64)
    n = offsets.shape[0] - 1
    roots = np.unique(np.atleast_1d(np.asarray(roots, dtype=np.int64)))
    bad = []
    if level.shape[0] != n:
        return ["level has wrong length"]
    # I1
    if roots.size and (level[roots] != 0).any():
        bad.append("I1: a root is not at level 0")
    zero = np.flatnonzero(level == 0)
    if zero.size != roots.size or (roots.size and not np.array_equal(np.sort(zero), roots)):
        bad.append("I1: level-0 set differs from the root set")
    if (level < -1).any():
        bad.append("level below -1")
    # I2
    deg = np.diff(offsets)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    lu, lv = level[src], level[cols]
    if ((lu == -1) != (lv == -1)).any():
        bad.append("I2: an edge joins a reached and an unreached vertex")
    both = (lu >= 0) & (lv >= 0)
    if (np.abs(lu[both] - lv[both]) > 1).any():
        bad.append("I2: an edge spans more than one level")
    # I3
    if parent is not None:
        parent = np.asarray(parent, dtype=np.int64)
        if roots.size and (parent[roots] != roots).any():
            bad.append("I1: a root's parent is not itself")
        if ((level == -1) & (parent != -1)).any():
            bad.append("I3: an unreached vertex has a parent")
        up = (lv >= 0) & (lv == lu - 1)          # edge src -> cols with cols one level up
        BIG = np.int64(1) << 40
        cand = np.where(up, cols, BIG)
        best = np.full(n, BIG, np.int64)
        nz = deg > 0
        if nz.any():
            red = np.minimum.reduceat(cand, offsets[:-1][nz]) if cand.size else np.zeros(0, np.int64)
            best[np.flatnonzero(nz)] = red
        inner = (level > 0)
        if (best[inner] >= BIG).any():
            bad.append("I3: a reached vertex has no neighbour one level up")
        if (parent[inner] != best[inner]).any():
            bad.append("I3: parent is not the smallest-id neighbour one level up")
    # I4
    lab = components(offsets, cols) if comp_labels is None else comp_labels
    want = np.isin(lab, lab[roots]) if roots.size else np.zeros(n, bool)
    if not np.array_equal(want, level >= 0):
        bad.append("I4: reached set differs from the roots' components")
    return bad
