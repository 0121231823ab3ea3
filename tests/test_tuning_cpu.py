"""Host logic of the autotuner front end: cache keys, storing and re-applying settings.
The library calls are replaced by recorders, so this runs without a GPU."""
import json
import types

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2209_08764_amd import _lib, tuning  # noqa: E402


class _Graph:
    def __init__(self, deg):
        self.offsets = torch.tensor(np.concatenate([[0], np.cumsum(deg)]), dtype=torch.int32)
        self.n = len(deg)
        self.m = int(np.sum(deg))


def _ws(deg, max_sources=256):
    return types.SimpleNamespace(graph=_Graph(deg), handle=1234, max_sources=max_sources)


@pytest.fixture
def calls(monkeypatch):
    rec = {"tune": [], "set": []}

    def fake_tune(handle, sources, what):
        rec["tune"].append((handle, list(sources), what))
        return {"batch_grain": 512, "batch_tile": 4096, "batch_levels": 4, "batch_pull": 99, "grid": 0,
                "small_edges": 4096, "push_edges": 7, "trials": 19, "default_ms": 2.0, "best_ms": 1.5}

    monkeypatch.setattr(tuning, "bfs_autotune", fake_tune)
    monkeypatch.setattr(tuning, "bfs_workspace_set_option", lambda h, o, v: rec["set"].append((h, o, v)))
    return rec


def test_signature_separates_graph_shapes():
    a = tuning.graph_signature(_Graph([1, 2, 0, 3]))
    assert a == "n=4,m=6,iso=1,dmax=3,d2=14"
    assert tuning.graph_signature(_Graph([2, 1, 0, 3])) == a          # same degree multiset
    assert tuning.graph_signature(_Graph([1, 2, 1, 2])) != a


def test_first_call_times_and_stores_then_reuses(calls, tmp_path):
    cache = str(tmp_path / "t.json")
    ws = _ws([1, 2, 0, 3])
    r1 = tuning.autotune(ws, [0, 1, 3], cache=cache)
    assert not r1["cached"] and calls["tune"] == [(1234, [0, 1, 3], _lib.BFS_TUNE_BATCH)]
    stored = json.load(open(cache))
    (key,) = stored
    assert f"|n=4,m=6,iso=1,dmax=3,d2=14|batch3|code={tuning.code_signature()}" in key
    r2 = tuning.autotune(_ws([1, 2, 0, 3]), [3, 1, 0], cache=cache)
    assert r2["cached"] and len(calls["tune"]) == 1
    applied = {o: v for _, o, v in calls["set"]}
    assert applied == {_lib.BFS_OPT_BATCH_GRAIN: 512, _lib.BFS_OPT_BATCH_TILE: 4096,
                       _lib.BFS_OPT_BATCH_LEVELS: 4, _lib.BFS_OPT_BATCH_PULL: 99}
    # another batch size or another graph is a different entry
    tuning.autotune(_ws([1, 2, 0, 3]), [0, 1], cache=cache)
    tuning.autotune(_ws([1, 2, 1, 2]), [0, 1, 3], cache=cache)
    assert len(calls["tune"]) == 3 and len(json.load(open(cache))) == 3


def test_single_source_kind_and_no_cache(calls):
    ws = _ws([1, 1], max_sources=1)
    r = tuning.autotune(ws, [0])
    assert not r["cached"] and calls["tune"][-1][2] == _lib.BFS_TUNE_SINGLE
    tuning.autotune(_ws([1, 1]), [0, 1], batch=False)
    assert calls["tune"][-1][2] == _lib.BFS_TUNE_SINGLE


def test_unreadable_cache_is_ignored(calls, tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    r = tuning.autotune(_ws([1, 2]), [0, 1], cache=str(p))
    assert not r["cached"] and len(json.load(open(p))) == 1


def test_code_signature_hashes_the_shipped_kernels():
    sig = tuning.code_signature()
    assert len(sig) == 12 and int(sig, 16) >= 0


def test_entries_of_other_kernel_code_are_timed_again(calls, tmp_path, monkeypatch):
    cache = str(tmp_path / "t.json")
    monkeypatch.setattr(tuning, "code_signature", lambda: "aaaaaaaaaaaa")
    tuning.autotune(_ws([1, 2, 0, 3]), [0, 1, 3], cache=cache)
    assert tuning.autotune(_ws([1, 2, 0, 3]), [0, 1, 3], cache=cache)["cached"]
    monkeypatch.setattr(tuning, "code_signature", lambda: "bbbbbbbbbbbb")
    assert not tuning.autotune(_ws([1, 2, 0, 3]), [0, 1, 3], cache=cache)["cached"]
    assert len(calls["tune"]) == 2 and len(json.load(open(cache))) == 2
