"""Helpers for the GPU parity tests (argument plumbing only)."""
import concurrent.futures
import os

import numpy as np

import oracle


def host_threads(cap: int = 16) -> int:
    """Host threads for oracle runs: the process's CPU share, at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def run_single(ws, source, want_parent=True):
    level, parent = ws.run(int(source), want_parent=want_parent)
    ws.sync()
    return level.cpu().numpy(), (parent.cpu().numpy() if parent is not None else None)


def assert_same(got_l, got_p, g, roots, want=None):
    """Element-by-element equality with the oracle (computed here unless `want` holds it)."""
    want_l, want_p = oracle.bfs(g.offsets, g.cols, roots) if want is None else want
    bad_l = np.flatnonzero(got_l != want_l)
    assert bad_l.size == 0, f"level differs at {bad_l[:10]}: got {got_l[bad_l[:10]]} want {want_l[bad_l[:10]]}"
    if got_p is not None:
        bad_p = np.flatnonzero(got_p != want_p)
        assert bad_p.size == 0, f"parent differs at {bad_p[:10]}: got {got_p[bad_p[:10]]} want {want_p[bad_p[:10]]}"
    return want_l, want_p


def oracle_many(g, sources, with_parent=True, threads=None):
    """oracle.bfs of each source, one source per host thread (the oracle is C code called
    through ctypes, which releases the interpreter lock), in the order of `sources`."""
    threads = threads or host_threads()

    def one(s):
        return oracle.bfs(g.offsets, g.cols, int(s), with_parent=with_parent)

    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as pool:
        return list(pool.map(one, list(sources)))


def oracle_batch_u8(g, sources, threads=None):
    """oracle.bfs_batch_u8 over `sources`, split into column blocks computed on host threads."""
    threads = threads or host_threads()
    sources = np.asarray(sources, np.int32)
    k = sources.size
    blocks = [sources[i:i + max(1, -(-k // threads))] for i in range(0, k, max(1, -(-k // threads)))]

    def one(b):
        return oracle.bfs_batch_u8(g.offsets, g.cols, b)

    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as pool:
        parts = list(pool.map(one, blocks))
    return np.concatenate([p[0] for p in parts], axis=1), any(p[1] for p in parts)
