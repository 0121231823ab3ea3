"""CPU oracle for the BFS library -- TEST INFRASTRUCTURE ONLY.

Only the tests, the harness smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never does, and this package never
imports the GPU library: the two share no code.  Inputs come from the
separate ``graphgen`` module, which holds no BFS arithmetic.

Contents
  oracle.c         plain sequential FIFO BFS and min-id parent pass (the
                   definition of Figure 1's output d[0:n-1], plus parents)
  brute.py         Floyd-Warshall all-pairs distances (a different algorithm)
  certify.py       O(n + m) certificate that a (level, parent) pair is exact
  s3bfs_steps.py   one search round as separate primitives (degree gather,
                   prefix sums, chunk starts, scanning, ownership filter,
                   concatenation; Figure 1 and the Algorithm and Analysis
                   paragraphs), the reference for the GPU primitives and the
                   per-level statistics
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# a differently built copy (e.g. a sanitizer build) may be loaded instead by naming it here
_LIB = os.environ.get("S3BFS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c (plain -O2, single-threaded, no intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
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
    lib.oracle_bfs_levels.restype = ctypes.c_int32
    lib.oracle_bfs_levels.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p, i32p]
    lib.oracle_parents.restype = None
    lib.oracle_parents.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p]
    lib.oracle_bfs.restype = ctypes.c_int32
    lib.oracle_bfs.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p, i32p, i32p]
    lib.oracle_bfs_batch_u8.restype = ctypes.c_int32
    lib.oracle_bfs_batch_u8.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, i32p,
                                        ctypes.POINTER(ctypes.c_uint8)]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _csr(offsets, cols):
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    if cols.size == 0:
        cols = np.zeros(1, np.int32)
    return offsets, cols


def bfs(offsets, cols, source, with_parent: bool = True):
    """(level, parent) from one source, or from several roots (nearest-root distance)."""
    offsets, cols = _csr(offsets, cols)
    n = offsets.shape[0] - 1
    roots = np.atleast_1d(np.asarray(source, dtype=np.int32)).copy()
    level = np.empty(max(n, 1), np.int32)[:n]
    parent = np.empty(max(n, 1), np.int32)[:n] if with_parent else None
    rc = _load().oracle_bfs(n, _p(offsets), _p(cols), roots.size, _p(roots), _p(level),
                            _p(parent) if with_parent else None)
    if rc == -1:
        raise ValueError("root out of range")
    if rc < 0:
        raise MemoryError("oracle out of memory")
    return (level, parent) if with_parent else level


def bfs_levels(offsets, cols, source):
    return bfs(offsets, cols, source, with_parent=False)


def parents(offsets, cols, level):
    offsets, cols = _csr(offsets, cols)
    n = offsets.shape[0] - 1
    level = np.ascontiguousarray(level, dtype=np.int32)
    parent = np.empty(n, np.int32)
    _load().oracle_parents(n, _p(offsets), _p(cols), _p(level), _p(parent))
    return parent


def bfs_batch_u8(offsets, cols, sources):
    """uint8 [n][k] levels of k single-source searches (255 = unreached); also the overflow flag."""
    offsets, cols = _csr(offsets, cols)
    n = offsets.shape[0] - 1
    sources = np.ascontiguousarray(sources, dtype=np.int32)
    k = sources.size
    out = np.empty((n, k), np.uint8)
    rc = _load().oracle_bfs_batch_u8(n, _p(offsets), _p(cols), k, _p(sources),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc < 0:
        raise ValueError("oracle batch failed (%d)" % rc)
    return out, bool(rc)


def level_stats(offsets, level):
    """Per-level frontier size n_l and frontier degree total e_l (the work
    accounting of the Analysis paragraph), from a level array."""
    level = np.asarray(level)
    deg = np.diff(np.asarray(offsets, dtype=np.int64))
    reached = level >= 0
    if not reached.any():
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    L = int(level[reached].max()) + 1
    n_l = np.bincount(level[reached], minlength=L).astype(np.int64)
    e_l = np.bincount(level[reached], weights=deg[reached], minlength=L).astype(np.int64)
    return n_l, e_l


def timed_bfs(offsets, cols, source):
    """Oracle BFS with the search and the parent pass timed separately (seconds)."""
    offsets, cols = _csr(offsets, cols)
    n = offsets.shape[0] - 1
    roots = np.atleast_1d(np.asarray(source, dtype=np.int32)).copy()
    level = np.empty(n, np.int32)
    parent = np.empty(n, np.int32)
    lib = _load()
    t0 = time.perf_counter()
    lib.oracle_bfs_levels(n, _p(offsets), _p(cols), roots.size, _p(roots), _p(level))
    t1 = time.perf_counter()
    lib.oracle_parents(n, _p(offsets), _p(cols), _p(level), _p(parent))
    t2 = time.perf_counter()
    return level, parent, t1 - t0, t2 - t1
