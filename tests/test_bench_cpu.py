"""bench.py's host-side measurement helpers on synthetic rocprofv3-shaped databases:
the copy calibration scales the counters, dispatch slices are taken in start order, and
the stored traffic is used only while the kernel source hash matches."""
import json
import os
import sqlite3
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _counters(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real, "
                "duration integer, dispatch_id integer)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?, ?)", rows)
    con.commit()
    return str(path)


def test_traffic_scaled_by_copy_calibration(tmp_path):
    k = "void k_persistent<false>(Params)"
    fetch = _counters(tmp_path / "f.db", [(k, "FETCH_SIZE", 1000.0, 1, 1), (k, "FETCH_SIZE", 3000.0, 1, 2),
                                          ("other", "FETCH_SIZE", 9e9, 1, 3)])
    write = _counters(tmp_path / "w.db", [(k, "WRITE_SIZE", 500.0, 1, 1), (k, "WRITE_SIZE", 500.0, 1, 2)])
    # the 1 GiB copy reads as half its size on FETCH_SIZE and its full size on WRITE_SIZE
    cf = _counters(tmp_path / "cf.db", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0, 1, 1)])
    cw = _counters(tmp_path / "cw.db", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0, 1, 1)])
    out = bench.traffic_from([fetch, write, cf, cw], out_dir=str(tmp_path))
    assert out["dispatches"] == 2
    assert out["copy_calibration"]["fetch_factor"] == 2.0 and out["copy_calibration"]["write_factor"] == 1.0
    assert out["hbm_fetch_bytes_per_launch"] == 2000 * 1024 * 2
    assert out["hbm_write_bytes_per_launch"] == 500 * 1024
    assert out["hbm_bytes_per_launch"] == 2000 * 1024 * 2 + 500 * 1024
    stored = json.load(open(tmp_path / "traffic_persistent_rmat24.json"))
    assert stored == out and stored["kernel_source_sha256_16"] == bench.kernel_source_hash()


def test_traffic_refuses_missing_kernel(tmp_path):
    empty = _counters(tmp_path / "e.db", [("other", "FETCH_SIZE", 1.0, 1, 1)])
    with pytest.raises(SystemExit):
        bench.traffic_from([empty, empty, empty, empty], out_dir=str(tmp_path))


def test_dispatch_slice_in_start_order(tmp_path, capsys):
    con = sqlite3.connect(tmp_path / "t.db")
    con.execute("create table kernels (name text, start integer, duration integer)")
    # durations 1..10 ms, inserted out of order
    rows = [("void k_persistent<false>(Params)", 100 * i, (i + 1) * 1_000_000) for i in range(10)]
    con.executemany("insert into kernels values (?, ?, ?)", rows[::-1] + [("k_prep", 5, 7)])
    con.commit()
    bench.rocpd_dispatches("k_persistent<false>", 3, 4, str(tmp_path / "t.db"))
    d = json.loads(capsys.readouterr().out)
    assert d["dispatches_total"] == 10 and d["taken"] == 4
    assert d["mean_ms"] == pytest.approx(np.mean([4, 5, 6, 7])) and d["min_ms"] == 4 and d["max_ms"] == 7


def test_stored_traffic_needs_matching_hash(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    path = tmp_path / "traffic_persistent_x.json"
    path.write_text(json.dumps({"kernel_source_sha256_16": "0" * 16, "hbm_bytes_per_launch": 5}))
    assert bench.stored_traffic("x") is None
    path.write_text(json.dumps({"kernel_source_sha256_16": bench.kernel_source_hash(), "hbm_bytes_per_launch": 5}))
    assert bench.stored_traffic("x") == 5


def test_algorithmic_bytes():
    run, kernel = bench.algorithmic_bytes(n=100, n_c=40, m_c=1000)
    assert run == 4 * 1000 + 8 * 100 + 16 * 40
    assert kernel == 4 * 1000 + 24 * 40


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("// note\nint f(int x) {\n    return x + 1;  /* one */\n}\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", [str(src)])
    h0 = bench.kernel_source_hash()
    src.write_text("// another note\nint f(int x) { return x + 1; }\n")
    assert bench.kernel_source_hash() == h0
    src.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != h0
