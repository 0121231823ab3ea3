"""S3BFS on one AMD Instinct MI355X: Python binding of libbfs.

The functions below carry the names of the C entry points in include/bfs.h
and only marshal arguments (torch tensors for device memory, torch streams
for ordering); the search itself runs in the library's HIP kernels.  The
classes ``Graph`` and ``Workspace`` are small conveniences over the same
calls that own the handles and the borrowed tensors.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (BFS_DEVICE_PTRS, BFS_HOST_PTRS, BFS_HOT_FILTER, BFS_LEAN, BFS_MODE_AUTO, BFS_MODE_DIRECTION,
                   BFS_MODE_INSENSITIVE, BFS_MODE_LEVEL, BFS_OPT_BU_ALPHA, BFS_OPT_BU_BETA, BFS_OPT_DENSE_EDGES,
                   BFS_MODE_PLAIN, BFS_OPT_BATCH_GRAIN, BFS_OPT_BATCH_LEVELS, BFS_OPT_BATCH_PULL, BFS_OPT_BATCH_TILE,
                   BFS_OPT_GRID, BFS_OPT_MODE, BFS_OPT_PROFILE, BFS_OPT_PUSH_EDGES, BFS_OPT_SMALL_EDGES,
                   BFS_OPT_BATCH_REPLAYS, BFS_OPT_GROUP, BFS_OPT_HOST_STATUS, BFS_OPT_SPLIT, BFS_TUNE_BATCH,
                   BFS_TUNE_SINGLE, BFS_VALIDATE, BFSError, bfs_stats_t, bfs_tune_t)

__all__ = [
    "bfs_init", "bfs_graph_free", "bfs_graph_info", "bfs_graph_aux_bytes", "bfs_workspace_bytes", "bfs_workspace_create",
    "bfs_workspace_free", "bfs_workspace_set_option", "bfs_workspace_grid_capacity", "bfs_run", "bfs_run_multiroot", "bfs_run_batch", "bfs_run_noalloc",
    "bfs_sync", "bfs_run_status", "bfs_last_stats", "bfs_last_level_stats", "bfs_last_level_times", "bfs_kernel_times", "bfs_status_str",
    "bfs_prim_compact",
    "bfs_prim_grain", "bfs_probe_rate_kernel", "bfs_autotune", "bfs_workspace_get_tuning", "Graph", "Workspace", "BFSError",
    "BFS_MODE_AUTO", "BFS_MODE_LEVEL", "BFS_MODE_PLAIN", "BFS_MODE_INSENSITIVE", "BFS_MODE_DIRECTION",
    "BFS_OPT_BU_ALPHA", "BFS_OPT_BU_BETA", "BFS_OPT_DENSE_EDGES", "BFS_OPT_MODE",
    "BFS_OPT_SMALL_EDGES", "BFS_OPT_GRID", "BFS_OPT_PROFILE", "BFS_OPT_BATCH_PULL", "BFS_OPT_PUSH_EDGES", "BFS_OPT_BATCH_LEVELS",
    "BFS_OPT_BATCH_GRAIN", "BFS_OPT_BATCH_TILE", "BFS_OPT_SPLIT", "BFS_OPT_GROUP", "BFS_OPT_BATCH_REPLAYS", "BFS_OPT_HOST_STATUS", "BFS_TUNE_BATCH", "BFS_TUNE_SINGLE", "BFS_HOST_PTRS",
    "BFS_DEVICE_PTRS", "BFS_VALIDATE", "BFS_HOT_FILTER", "BFS_LEAN",
]


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _dptr(t, dtype, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous {dtype} tensor")
    return t.data_ptr() if t.numel() else None


def bfs_status_str(status: int) -> str:
    return _lib.load().bfs_status_str(status).decode()


def bfs_init(offsets, cols, flags: int | None = None, stream=None, validate: bool = False,
             hot: bool | None = None, sort_rows: bool = False) -> int:
    """Make a CSR graph resident; numpy arrays are copied, device tensors borrowed.
    hot: None = the library's size rule for the hot-vertex filter, True/False = force it on/off.
    sort_rows: rows need not be sorted; the library sorts a copy (BFS_SORT_ROWS)."""
    torch = _torch()
    lib = _lib.load()
    out = ctypes.c_void_p()
    if isinstance(offsets, torch.Tensor) and offsets.is_cuda:
        n = offsets.numel() - 1
        m = cols.numel()
        fl = BFS_DEVICE_PTRS if flags is None else flags
        po = _dptr(offsets, torch.int32, "offsets")
        pc = _dptr(cols, torch.int32, "cols") if m else None
    else:
        offsets = np.ascontiguousarray(offsets, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        n = offsets.size - 1
        m = cols.size
        fl = BFS_HOST_PTRS if flags is None else flags
        po = offsets.ctypes.data
        pc = cols.ctypes.data if m else None
    if validate:
        fl |= BFS_VALIDATE
    if hot is not None:
        fl |= BFS_HOT_FILTER if hot else BFS_LEAN
    if sort_rows:
        fl |= _lib.BFS_SORT_ROWS
    _lib.check(lib.bfs_init(po, pc, n, m, fl, _stream_ptr(stream), ctypes.byref(out)), "bfs_init")
    return out.value


def bfs_graph_free(g: int) -> None:
    _lib.check(_lib.load().bfs_graph_free(g), "bfs_graph_free")


def bfs_graph_info(g: int):
    n = ctypes.c_int32()
    m = ctypes.c_int64()
    _lib.check(_lib.load().bfs_graph_info(g, ctypes.byref(n), ctypes.byref(m)), "bfs_graph_info")
    return n.value, m.value


def bfs_graph_aux_bytes(g: int) -> int:
    return int(_lib.load().bfs_graph_aux_bytes(g))


def bfs_workspace_bytes(g: int, max_sources: int = 1) -> int:
    return int(_lib.load().bfs_workspace_bytes(g, max_sources))


def bfs_workspace_create(g: int, max_sources: int = 1) -> int:
    out = ctypes.c_void_p()
    _lib.check(_lib.load().bfs_workspace_create(g, max_sources, ctypes.byref(out)), "bfs_workspace_create")
    return out.value


def bfs_workspace_free(ws: int) -> None:
    _lib.check(_lib.load().bfs_workspace_free(ws), "bfs_workspace_free")


def bfs_workspace_set_option(ws: int, option: int, value: int) -> None:
    _lib.check(_lib.load().bfs_workspace_set_option(ws, option, int(value)), "bfs_workspace_set_option")


def bfs_workspace_grid_capacity(ws: int) -> int:
    return int(_lib.load().bfs_workspace_grid_capacity(ws))


def bfs_run(ws: int, source: int, level, parent=None, stream=None) -> None:
    torch = _torch()
    pl = _dptr(level, torch.int32, "level")
    pp = _dptr(parent, torch.int32, "parent") if parent is not None else None
    _lib.check(_lib.load().bfs_run(ws, int(source), pl, pp, _stream_ptr(stream)), "bfs_run")


def bfs_run_multiroot(ws: int, roots, level, parent=None, stream=None) -> None:
    torch = _torch()
    roots = np.ascontiguousarray(roots, dtype=np.int32)
    pl = _dptr(level, torch.int32, "level")
    pp = _dptr(parent, torch.int32, "parent") if parent is not None else None
    _lib.check(_lib.load().bfs_run_multiroot(ws, roots.ctypes.data, roots.size, pl, pp, _stream_ptr(stream)),
               "bfs_run_multiroot")


def bfs_run_batch(ws: int, sources, level, stream=None) -> None:
    torch = _torch()
    sources = np.ascontiguousarray(sources, dtype=np.int32)
    pl = _dptr(level, torch.uint8, "level")
    _lib.check(_lib.load().bfs_run_batch(ws, sources.ctypes.data, sources.size, pl, _stream_ptr(stream)),
               "bfs_run_batch")


def bfs_run_noalloc(g: int, source: int, level, parent=None, status=None, stream=None) -> None:
    """Single-source search on graph handle g from the library's static scratch (allocates nothing)."""
    torch = _torch()
    pl = _dptr(level, torch.int32, "level")
    pp = _dptr(parent, torch.int32, "parent") if parent is not None else None
    ps = _dptr(status, torch.int32, "status") if status is not None else None
    _lib.check(_lib.load().bfs_run_noalloc(g, int(source), pl, pp, ps, _stream_ptr(stream)), "bfs_run_noalloc")


def bfs_sync(ws: int) -> None:
    _lib.check(_lib.load().bfs_sync(ws), "bfs_sync")


def bfs_run_status(ws: int) -> int:
    """Device status of the last run (needs BFS_OPT_HOST_STATUS); BFSError(BFS_EBUSY) while it runs."""
    st = ctypes.c_int32()
    _lib.check(_lib.load().bfs_run_status(ws, ctypes.byref(st)), "bfs_run_status")
    return int(st.value)


def bfs_last_stats(ws: int) -> dict:
    st = bfs_stats_t()
    _lib.check(_lib.load().bfs_last_stats(ws, ctypes.byref(st)), "bfs_last_stats")
    return {f: getattr(st, f) for f, _ in bfs_stats_t._fields_}


def bfs_last_level_stats(ws: int, cap: int = 1 << 16):
    n_l = np.zeros(cap, np.int64)
    e_l = np.zeros(cap, np.int64)
    cnt = ctypes.c_int32()
    _lib.check(_lib.load().bfs_last_level_stats(ws, cap, n_l.ctypes.data, e_l.ctypes.data, ctypes.byref(cnt)),
               "bfs_last_level_stats")
    return n_l[:cnt.value].copy(), e_l[:cnt.value].copy()


def bfs_last_level_times(ws: int, cap: int = 1 << 16):
    ex = np.zeros(cap, np.float64)
    co = np.zeros(cap, np.float64)
    cnt = ctypes.c_int32()
    _lib.check(_lib.load().bfs_last_level_times(ws, cap, ex.ctypes.data, co.ctypes.data, ctypes.byref(cnt)),
               "bfs_last_level_times")
    return ex[:cnt.value].copy(), co[:cnt.value].copy()


def bfs_kernel_times(ws: int, cap: int = 4096) -> np.ndarray:
    ms = np.zeros(cap, np.float64)
    cnt = ctypes.c_int32()
    _lib.check(_lib.load().bfs_kernel_times(ws, cap, ms.ctypes.data, ctypes.byref(cnt)), "bfs_kernel_times")
    return ms[:cnt.value].copy()


def bfs_prim_grain() -> int:
    return int(_lib.load().bfs_prim_grain())


def bfs_prim_compact(offsets, owner, cand, cnt, out_v, out_rs, out_ex, out_tstart, totals, stream=None) -> None:
    torch = _torch()
    i32 = torch.int32
    _lib.check(_lib.load().bfs_prim_compact(
        _dptr(offsets, i32, "offsets"), offsets.numel() - 1, _dptr(owner, i32, "owner"), _dptr(cand, i32, "cand"),
        _dptr(cnt, i32, "cnt"), cnt.numel(), _dptr(out_v, i32, "out_v"), _dptr(out_rs, i32, "out_rs"),
        _dptr(out_ex, i32, "out_ex"),
        _dptr(out_tstart, i32, "out_tstart"), out_tstart.numel(), _dptr(totals, i32, "totals"), _stream_ptr(stream)),
        "bfs_prim_compact")


def bfs_probe_rate_kernel(idx, table, shift: int, sink, stream=None) -> None:
    """Launch the random-probe measurement kernel (asynchronous on stream)."""
    torch = _torch()
    _lib.check(_lib.load().bfs_probe_rate_kernel(
        _dptr(idx, torch.int32, "idx"), idx.numel(), _dptr(table, torch.int32, "table"), table.numel(), int(shift),
        _dptr(sink, torch.int32, "sink"), _stream_ptr(stream)), "bfs_probe_rate_kernel")


def bfs_autotune(ws: int, sources, what: int) -> dict:
    """Time candidate launch settings on the workspace's graph and keep the fastest (synchronous)."""
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
    out = bfs_tune_t()
    _lib.check(_lib.load().bfs_autotune(ws, src.ctypes.data, int(src.size), int(what), ctypes.byref(out)),
               "bfs_autotune")
    return out.as_dict()


def bfs_workspace_get_tuning(ws: int) -> dict:
    out = bfs_tune_t()
    _lib.check(_lib.load().bfs_workspace_get_tuning(ws, ctypes.byref(out)), "bfs_workspace_get_tuning")
    return out.as_dict()


class Graph:
    """A device-resident graph (owns the handle and keeps borrowed tensors alive)."""

    def __init__(self, offsets, cols, device="cuda", validate: bool = False, copy: bool = False,
                 hot: bool | None = None, sort_rows: bool = False):
        torch = _torch()
        if isinstance(offsets, np.ndarray) and not copy:
            offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int32)).to(device)
            cols = torch.from_numpy(np.ascontiguousarray(cols, dtype=np.int32)).to(device)
        self._keep = (offsets, cols)
        self.handle = bfs_init(offsets, cols, validate=validate, hot=hot, sort_rows=sort_rows)
        self.n, self.m = bfs_graph_info(self.handle)
        self.aux_bytes = bfs_graph_aux_bytes(self.handle)
        self.offsets = offsets
        self.cols = cols

    def free(self):
        if self.handle:
            bfs_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Workspace:
    """Scratch for one in-flight run on a Graph."""

    def __init__(self, graph: Graph, max_sources: int = 1, mode: int | None = None, **opts):
        self.graph = graph
        self.max_sources = max_sources
        self.handle = bfs_workspace_create(graph.handle, max_sources)
        if mode is not None:
            bfs_workspace_set_option(self.handle, BFS_OPT_MODE, mode)
        names = {"small_edges": BFS_OPT_SMALL_EDGES, "grid": BFS_OPT_GRID, "profile": BFS_OPT_PROFILE,
                 "batch_pull": BFS_OPT_BATCH_PULL, "push_edges": BFS_OPT_PUSH_EDGES,
                 "batch_levels": BFS_OPT_BATCH_LEVELS, "batch_grain": BFS_OPT_BATCH_GRAIN,
                 "batch_tile": BFS_OPT_BATCH_TILE, "bu_alpha": BFS_OPT_BU_ALPHA, "bu_beta": BFS_OPT_BU_BETA,
                 "dense_edges": BFS_OPT_DENSE_EDGES, "split_search": BFS_OPT_SPLIT, "group": BFS_OPT_GROUP,
                 "batch_replays": BFS_OPT_BATCH_REPLAYS, "host_status": BFS_OPT_HOST_STATUS}
        for k, v in opts.items():
            bfs_workspace_set_option(self.handle, names[k], v)

    def set(self, option: int, value: int):
        bfs_workspace_set_option(self.handle, option, value)

    def run(self, source: int, level=None, parent=None, stream=None, want_parent: bool = True):
        torch = _torch()
        n = self.graph.n
        if level is None:
            level = torch.empty(n, dtype=torch.int32, device="cuda")
        if parent is None and want_parent:
            parent = torch.empty(n, dtype=torch.int32, device="cuda")
        bfs_run(self.handle, source, level, parent, stream)
        return level, parent

    def run_multiroot(self, roots, level=None, parent=None, stream=None):
        torch = _torch()
        n = self.graph.n
        if level is None:
            level = torch.empty(n, dtype=torch.int32, device="cuda")
        if parent is None:
            parent = torch.empty(n, dtype=torch.int32, device="cuda")
        bfs_run_multiroot(self.handle, roots, level, parent, stream)
        return level, parent

    def run_batch(self, sources, level=None, stream=None):
        torch = _torch()
        k = len(sources)
        if level is None:
            level = torch.empty(self.graph.n * k, dtype=torch.uint8, device="cuda")
        bfs_run_batch(self.handle, sources, level, stream)
        return level

    def sync(self):
        bfs_sync(self.handle)

    def run_status(self) -> int:
        return bfs_run_status(self.handle)

    def tuning(self) -> dict:
        return bfs_workspace_get_tuning(self.handle)

    def autotune(self, sources, batch: bool | None = None, cache: str | None = None) -> dict:
        """Pick launch settings for this graph (see tuning.autotune); returns them."""
        from .tuning import autotune
        return autotune(self, sources, batch=batch, cache=cache)

    def stats(self):
        return bfs_last_stats(self.handle)

    def grid_capacity(self) -> int:
        return bfs_workspace_grid_capacity(self.handle)

    def level_stats(self, cap: int = 1 << 16):
        return bfs_last_level_stats(self.handle, cap)

    def kernel_times(self):
        return bfs_kernel_times(self.handle)

    def level_times(self, cap: int = 1 << 16):
        return bfs_last_level_times(self.handle, cap)

    def free(self):
        if self.handle:
            bfs_workspace_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
