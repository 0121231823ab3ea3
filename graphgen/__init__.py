"""Seeded synthetic graph generators shared by the oracle tests and the GPU library.

This module is input generation only: it builds symmetric CSR graphs
(``int32 offsets[n+1]``, ``int32 cols[m]``, rows sorted ascending, no
self-loops, no duplicates) and seeded source lists.  It computes no part of
a breadth-first search.  The paper evaluates on a Wikipedia graph and on
unnamed real-world and synthetic graphs (Experimental Results); the seeded
R-MAT, grid, Erdos-Renyi and forest graphs built here stand in for them.

The heavy lifting is in ``gen.c`` (OpenMP, counter-based randomness, so the
output does not depend on the thread count); ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
# a differently built copy (e.g. a sanitizer build) may be loaded instead by naming it here
_LIB = os.environ.get("S3BFS_GRAPHGEN_LIB") or os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def build(force: bool = True) -> str:
    """Compile gen.c into libgraphgen.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.gg_draw.restype = ctypes.c_uint64
    lib.gg_draw.argtypes = [ctypes.c_uint64] * 3
    lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, i32p]
    lib.gg_rmat_samples.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, i32p, i32p]
    lib.gg_er_samples.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
    lib.gg_forest_samples.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, i32p, i32p]
    lib.gg_csr_build.restype = ctypes.c_int64
    lib.gg_csr_build.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, ctypes.POINTER(ctypes.c_void_p)]
    lib.gg_csr_emit.restype = ctypes.c_int
    lib.gg_csr_emit.argtypes = [ctypes.c_void_p, i32p, i32p]
    lib.gg_grid_m.restype = ctypes.c_int64
    lib.gg_grid_m.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, i32p]
    lib.gg_pick_sources.restype = ctypes.c_int64
    lib.gg_pick_sources.argtypes = [ctypes.c_int32, i32p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int, i32p]
    lib.gg_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class Graph:
    """A symmetric CSR graph with the recipe that produced it."""

    offsets: np.ndarray
    cols: np.ndarray
    name: str = "graph"
    recipe: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.cols.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)


def draw(seed: int, stream: int, counter: int) -> int:
    return int(_load().gg_draw(seed, stream, counter))


def permutation(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, np.int32)
    _load().gg_permutation(n, seed, _p(out))
    return out


def csr_from_pairs(n: int, src: np.ndarray, dst: np.ndarray, name="pairs", recipe=None) -> Graph:
    """Symmetric, sorted, deduplicated CSR without self-loops from edge samples."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    assert src.shape == dst.shape
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    work = ctypes.c_void_p()
    m = lib.gg_csr_build(n, src.size, _p(src), _p(dst), ctypes.byref(work))
    if m > np.iinfo(np.int32).max:
        lib.gg_csr_emit(work, None, None)
        raise ValueError("graph too large for int32 CSR")
    offsets = np.empty(n + 1, np.int32)
    cols = np.empty(max(m, 0), np.int32)
    rc = lib.gg_csr_emit(work, _p(offsets), _p(cols) if m > 0 else _p(np.empty(1, np.int32)))
    if rc != 0:
        raise ValueError("graph too large for int32 CSR")
    return Graph(offsets, cols, name, dict(recipe or {}))


def rmat(scale: int, edgefactor: int = 16, abcd=RMAT_ABCD, seed: int = 1, permute: bool = True,
         perm_seed: int | None = None) -> Graph:
    """R-MAT graph, symmetrised and deduplicated, with a seeded vertex permutation."""
    a, b, c, d = abcd
    n = 1 << scale
    M = edgefactor * n
    src = np.empty(M, np.int32)
    dst = np.empty(M, np.int32)
    ps = seed ^ 0x5EED if perm_seed is None else perm_seed
    _load().gg_rmat_samples(scale, edgefactor, a, b, c, seed, int(permute), ps, _p(src), _p(dst))
    recipe = dict(kind="rmat", scale=scale, edgefactor=edgefactor, abcd=list(abcd), seed=seed,
                  permute=bool(permute), perm_seed=ps)
    g = csr_from_pairs(n, src, dst, name=f"rmat{scale}", recipe=recipe)
    del src, dst
    return g


def grid(W: int, H: int | None = None) -> Graph:
    """W x H 4-neighbour grid, vertex id = r * W + c."""
    H = W if H is None else H
    lib = _load()
    m = lib.gg_grid_m(W, H)
    offsets = np.empty(W * H + 1, np.int32)
    cols = np.empty(m, np.int32)
    lib.gg_grid(W, H, _p(offsets), _p(cols) if m > 0 else _p(np.empty(1, np.int32)))
    return Graph(offsets, cols, f"grid{W}x{H}", dict(kind="grid", W=W, H=H))


def erdos_renyi(n: int, mean_degree: float, seed: int = 1) -> Graph:
    """G(n, M) with M = mean_degree * n / 2 uniform pairs (before dedup)."""
    M = int(round(mean_degree * n / 2))
    src = np.empty(M, np.int32)
    dst = np.empty(M, np.int32)
    _load().gg_er_samples(n, M, seed, _p(src), _p(dst))
    return csr_from_pairs(n, src, dst, name=f"er{n}", recipe=dict(kind="er", n=n, mean_degree=mean_degree,
                                                                       seed=seed))


def powerlaw_forest(n: int, nroots: int = 64, seed: int = 1) -> Graph:
    """Preferential-attachment forest with nroots trees."""
    E = max(n - nroots, 0)
    src = np.empty(max(E, 1), np.int32)
    dst = np.empty(max(E, 1), np.int32)
    _load().gg_forest_samples(n, nroots, seed, _p(src), _p(dst))
    return csr_from_pairs(n, src[:E], dst[:E], name=f"forest{n}",
                          recipe=dict(kind="forest", n=n, nroots=nroots, seed=seed))


def from_edges(n: int, edges, name="edges") -> Graph:
    """Symmetric CSR from a list of (u, v) pairs (small hand-made graphs)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return csr_from_pairs(n, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), name=name,
                          recipe=dict(kind="edges"))


def pick_sources(g: Graph, k: int, seed: int = 1, distinct: bool = True) -> np.ndarray:
    """k sources uniform among vertices of degree >= 1 (without replacement if distinct)."""
    out = np.empty(max(k, 1), np.int32)
    ne = _load().gg_pick_sources(g.n, _p(g.offsets), seed, k, int(distinct), _p(out))
    if ne < 0:
        raise ValueError("not enough non-isolated vertices")
    return out[:k].copy()


def disjoint_union(graphs) -> tuple[Graph, np.ndarray]:
    """Disjoint union of graphs; returns the union and each part's first vertex id."""
    offs, colss, base = [], [], []
    vbase = 0
    ebase = 0
    for g in graphs:
        base.append(vbase)
        offs.append(g.offsets[:-1].astype(np.int64) + ebase)
        colss.append(g.cols.astype(np.int64) + vbase)
        vbase += g.n
        ebase += g.m
    if ebase > np.iinfo(np.int32).max or vbase > np.iinfo(np.int32).max:
        raise ValueError("union too large for int32 CSR")
    offsets = np.concatenate(offs + [np.array([ebase])]).astype(np.int32)
    cols = (np.concatenate(colss) if colss else np.empty(0)).astype(np.int32)
    return Graph(offsets, cols, "union", dict(kind="union", parts=len(base))), np.asarray(base, np.int32)


def num_threads() -> int:
    return int(_load().gg_num_threads())
