"""ctypes binding of libbfs (the C ABI in include/bfs.h).

Argument marshalling only: every step of the search runs in the library's
HIP kernels.  torch is used for device memory and streams.  If libbfs.so is
missing the import fails loudly; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfs.so")

BFS_OK = 0
BFS_EINVAL = -1
BFS_ERANGE = -2
BFS_ENOMEM = -3
BFS_EBADCSR = -4
BFS_EHIP = -5
BFS_EOVERFLOW = -6
BFS_EBUSY = -7
BFS_EDEVICE = -8

BFS_HOST_PTRS = 1
BFS_DEVICE_PTRS = 2
BFS_VALIDATE = 4
BFS_HOT_FILTER = 8
BFS_LEAN = 16
BFS_SORT_ROWS = 32

BFS_MODE_AUTO = 0
BFS_MODE_LEVEL = 1
BFS_MODE_PLAIN = 2
BFS_MODE_INSENSITIVE = 3
BFS_MODE_DIRECTION = 4

BFS_OPT_MODE = 1
BFS_OPT_SMALL_EDGES = 2
BFS_OPT_GRID = 3
BFS_OPT_PROFILE = 4
BFS_OPT_BATCH_PULL = 5
BFS_OPT_PUSH_EDGES = 6
BFS_OPT_BATCH_LEVELS = 7
BFS_OPT_BATCH_GRAIN = 8
BFS_OPT_BATCH_TILE = 9
BFS_OPT_BU_ALPHA = 10
BFS_OPT_BU_BETA = 11
BFS_OPT_DENSE_EDGES = 12
BFS_OPT_SPLIT = 13
BFS_OPT_GROUP = 14
BFS_OPT_BATCH_REPLAYS = 15
BFS_OPT_HOST_STATUS = 16

BFS_TUNE_BATCH = 1
BFS_TUNE_SINGLE = 2

MODE_NAMES = {BFS_MODE_AUTO: "auto", BFS_MODE_LEVEL: "level", BFS_MODE_PLAIN: "plain",
              BFS_MODE_INSENSITIVE: "insensitive", BFS_MODE_DIRECTION: "direction"}


class bfs_stats_t(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("small_levels", ctypes.c_int32),
        ("reached", ctypes.c_int64),
        ("edges", ctypes.c_int64),
        ("kernel_ms", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("stats_truncated", ctypes.c_int32),
        ("bottom_up_levels", ctypes.c_int32),
    ]


class bfs_tune_t(ctypes.Structure):
    _fields_ = [
        ("batch_grain", ctypes.c_int32),
        ("batch_tile", ctypes.c_int32),
        ("batch_levels", ctypes.c_int32),
        ("batch_pull", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("small_edges", ctypes.c_int32),
        ("push_edges", ctypes.c_int32),
        ("dense_edges", ctypes.c_int32),
        ("trials", ctypes.c_int32),
        ("default_ms", ctypes.c_double),
        ("best_ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class BFSError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func} failed with status {status}: {msg}")
        self.status = status


_lib = None

_SIGS = {
    "bfs_init": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "bfs_graph_free": (ctypes.c_int32, [ctypes.c_void_p]),
    "bfs_graph_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "bfs_graph_aux_bytes": (ctypes.c_int64, [ctypes.c_void_p]),
    "bfs_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int32]),
    "bfs_workspace_create": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "bfs_workspace_free": (ctypes.c_int32, [ctypes.c_void_p]),
    "bfs_workspace_set_option": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64]),
    "bfs_workspace_grid_capacity": (ctypes.c_int32, [ctypes.c_void_p]),
    "bfs_run": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]),
    "bfs_run_multiroot": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "bfs_run_batch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "bfs_run_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "bfs_sync": (ctypes.c_int32, [ctypes.c_void_p]),
    "bfs_last_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(bfs_stats_t)]),
    "bfs_last_level_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_int32)]),
    "bfs_kernel_times": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int32)]),
    "bfs_last_level_times": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_int32)]),
    "bfs_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "bfs_last_error": (ctypes.c_char_p, []),
    "bfs_prim_compact": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "bfs_prim_grain": (ctypes.c_int32, []),
    "bfs_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                                      ctypes.POINTER(bfs_tune_t)]),
    "bfs_workspace_get_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(bfs_tune_t)]),
    "bfs_probe_rate_kernel": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                               ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "bfs_workspace_set_spin_ticks": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64]),
    "bfs_run_status": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
}

EXPORTED = tuple(_SIGS)


def load(path: str = LIB_PATH):
    """Load libbfs.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libbfs.so not found at {path}; build it with python -m paper_2209_08764_amd._build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status: int, func: str) -> int:
    if status != BFS_OK:
        lib = load()
        raise BFSError(status, func, (lib.bfs_last_error() or b"").decode() or
                       lib.bfs_status_str(status).decode())
    return status
