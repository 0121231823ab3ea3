"""The C-ABI library loads on a machine without a GPU and exports every symbol that
include/*.h declares."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in ("bfs.h", "bfs_test.h")]
LIB = os.path.join(ROOT, "paper_2209_08764_amd", "libbfs.so")


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bfs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for want in ["bfs_init", "bfs_graph_free", "bfs_workspace_bytes", "bfs_workspace_create",
                 "bfs_workspace_free", "bfs_run", "bfs_run_batch", "bfs_run_multiroot", "bfs_last_stats",
                 "bfs_status_str", "bfs_sync"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libbfs.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_every_header_is_covered():
    assert sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))) == sorted(HEADERS)


def test_binding_covers_the_header():
    from paper_2209_08764_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions()


def test_status_strings_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libbfs.so not built")
    from paper_2209_08764_amd import _lib
    lib = _lib.load()
    assert lib.bfs_status_str(0) == b"ok"
    assert lib.bfs_status_str(-6) == b"batched level reached 255"
    # argument errors are reported before any device work
    assert lib.bfs_run(None, 0, None, None, None) == _lib.BFS_EINVAL
    assert lib.bfs_init(None, None, 0, 0, 1, None, None) == _lib.BFS_EINVAL
    assert b"null" in lib.bfs_last_error()
