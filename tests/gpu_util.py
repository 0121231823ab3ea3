"""Helpers for the GPU parity tests (argument plumbing only)."""
import numpy as np

import oracle


def run_single(ws, source, want_parent=True):
    level, parent = ws.run(int(source), want_parent=want_parent)
    ws.sync()
    return level.cpu().numpy(), (parent.cpu().numpy() if parent is not None else None)


def assert_same(got_l, got_p, g, roots):
    want_l, want_p = oracle.bfs(g.offsets, g.cols, roots)
    bad_l = np.flatnonzero(got_l != want_l)
    assert bad_l.size == 0, f"level differs at {bad_l[:10]}: got {got_l[bad_l[:10]]} want {want_l[bad_l[:10]]}"
    if got_p is not None:
        bad_p = np.flatnonzero(got_p != want_p)
        assert bad_p.size == 0, f"parent differs at {bad_p[:10]}: got {got_p[bad_p[:10]]} want {want_p[bad_p[:10]]}"
    return want_l, want_p
