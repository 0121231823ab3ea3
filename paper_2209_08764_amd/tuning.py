"""Autotuner front end: a persistent cache over bfs_autotune.

The search itself runs in the library (bfs_autotune times real runs of the
workspace's graph and keeps the fastest settings).  This module only
remembers the outcome per (device, graph shape, batch size, kernel code) in
a JSON file, so a later process applies the stored settings without timing
anything.  Settings never change results, only speed, so a stale or
mismatched entry costs time at worst.
"""
from __future__ import annotations

import functools
import hashlib
import json
import os

from . import (BFS_OPT_BATCH_GRAIN, BFS_OPT_BATCH_LEVELS, BFS_OPT_BATCH_PULL, BFS_OPT_BATCH_TILE, BFS_OPT_GRID,
               BFS_OPT_DENSE_EDGES, BFS_OPT_PUSH_EDGES, BFS_OPT_SMALL_EDGES, BFS_TUNE_BATCH, BFS_TUNE_SINGLE, bfs_autotune,
               bfs_workspace_set_option)

_BATCH_KEYS = {"batch_grain": BFS_OPT_BATCH_GRAIN, "batch_tile": BFS_OPT_BATCH_TILE,
               "batch_pull": BFS_OPT_BATCH_PULL, "batch_levels": BFS_OPT_BATCH_LEVELS}
_SINGLE_KEYS = {"grid": BFS_OPT_GRID, "small_edges": BFS_OPT_SMALL_EDGES, "push_edges": BFS_OPT_PUSH_EDGES,
                "dense_edges": BFS_OPT_DENSE_EDGES}


def graph_signature(graph) -> str:
    """Shape of a device graph: n, m, isolated count, maximum degree and the degree second moment."""
    import torch
    deg = torch.diff(graph.offsets.to(torch.int64))
    iso = int((deg == 0).sum())
    mx = int(deg.max()) if deg.numel() else 0
    m2 = int((deg * deg).sum()) if deg.numel() else 0
    return f"n={graph.n},m={graph.m},iso={iso},dmax={mx},d2={m2}"


def device_signature() -> str:
    """The GPU a tuning applies to: its architecture and compute-unit count (the marketing name
    is not always readable)."""
    import torch
    if not torch.cuda.is_available():
        return "cpu"
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "") or torch.cuda.get_device_name()
    return f"{arch.split(':')[0]}/{props.multi_processor_count}cu"


_KERNEL_SOURCES = ("bfs_kernels.hip", "bfs_batch.hip", "bfs_device.h", "bfs_internal.h")


@functools.lru_cache(maxsize=1)
def code_signature() -> str:
    """The kernels a tuning is timed with: a hash of their sources as the package ships them
    (empty without them), so that settings tuned for other kernels are timed again."""
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for name in _KERNEL_SOURCES:
        try:
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
        except OSError:
            return ""
    return h.hexdigest()[:12]


def cache_key(ws, k: int, batch: bool) -> str:
    kind = f"batch{k}" if batch else "single"
    code = code_signature()
    return f"{device_signature()}|{graph_signature(ws.graph)}|{kind}" + (f"|code={code}" if code else "")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def apply(ws, entry: dict, batch: bool) -> None:
    keys = _BATCH_KEYS if batch else _SINGLE_KEYS
    for name, opt in keys.items():
        if name in entry:
            bfs_workspace_set_option(ws.handle, opt, int(entry[name]))


def autotune(ws, sources, batch: bool | None = None, cache: str | None = None) -> dict:
    """Tune ws for runs like `sources` (one batch of them, or each single-source).

    With `cache` (a JSON path), a stored entry for the same device, graph
    shape and batch size is applied instead of timing; otherwise the result
    of the timing is stored there.  Returns the settings in force, plus
    "cached": True/False.
    """
    sources = list(int(s) for s in sources)
    if batch is None:
        batch = len(sources) > 1 and ws.max_sources > 1
    key = cache_key(ws, len(sources), batch) if cache else None
    if cache:
        entry = _load(cache).get(key)
        if entry:
            apply(ws, entry, batch)
            return dict(entry, cached=True)
    res = bfs_autotune(ws.handle, sources, BFS_TUNE_BATCH if batch else BFS_TUNE_SINGLE)
    if cache:
        table = _load(cache)
        table[key] = res
        tmp = f"{cache}.tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(res, cached=False)
