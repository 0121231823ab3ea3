#!/usr/bin/env python3
"""Benchmark of the S3BFS hot path on one MI355X.

Headline workload: R-MAT scale 24 (edge factor 16, a/b/c/d = .57/.19/.19/.05,
symmetrised, deduplicated, vertex-permuted), 64 seeded sources run one at a
time.  One "step" is one pass over all 64 sources, each a complete
single-source search (init, every level, parents); `value` is the harmonic
mean over the sources of GTEPS = (undirected edges in the source's
component) / (median time of its search over the steps), with the CSR
already resident in HBM.  The oracle's answers for the CPU-baseline sample
are compared with the GPU's (extras.parity_*).

Printed on one JSON line: the contract fields, a roofline object for the
dominant kernel (the persistent level-loop kernel, timed with HIP events on
its stream), the CPU oracle's throughput on a bounded sample, and extras
(the plain per-level kernel, per-level launches and the work-insensitive
variant on the same graph; the other workloads when implemented).
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GTEPS single-source & 256-source batch vs plain; p50/p99 query latency"
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SRC = [os.path.join(ROOT, "paper_2209_08764_amd", "csrc", f)
              for f in ("bfs_kernels.hip", "bfs_device.h", "bfs_internal.h")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def hmean(x):
    x = np.asarray(x, dtype=np.float64)
    return float(len(x) / np.sum(1.0 / x)) if len(x) else float("nan")


def kernel_source_hash() -> str:
    """Hash of the search kernel's code (the kernel file and the device headers it includes).
    Comments and layout are left out, so that stored counters stay valid across comment edits
    and go stale with any change to the code itself."""
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        text = open(path, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def algorithmic_bytes(n: int, n_c: int, m_c: int):
    """Bytes the search must move at least once: each reached row's columns (4 m_c), level and
    parent of every vertex (8 n), and per reached vertex its offsets pair and one frontier
    write and read (16 n_c).  The search kernel's share leaves out the -1 fill of unreached
    vertices, which the preparation kernel does: 4 m_c + 8 n_c + 16 n_c."""
    run = 4 * m_c + 8 * n + 16 * n_c
    kernel = 4 * m_c + 24 * n_c
    return run, kernel


def stored_traffic(workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they match this kernel source."""
    path = os.path.join(PROFILE_DIR, f"traffic_persistent_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def time_passes(ws, level, parent, sources, passes, torch):
    """`passes` complete passes over the workload's sources, each search bracketed by HIP
    events on the current stream.  Returns per-search ms [passes][len(sources)], the wall
    ms of all passes, and the search kernel's own durations (profiled runs)."""
    from paper_2209_08764_amd import bfs_kernel_times, bfs_run
    ws_h = ws.handle
    k = len(sources)
    if passes * k > 4096:
        raise ValueError("at most 4096 profiled searches per measurement (lower --steps)")
    bfs_kernel_times(ws_h)  # forget earlier profiled runs
    starts = [[torch.cuda.Event(enable_timing=True) for _ in range(k)] for _ in range(passes)]
    ends = [[torch.cuda.Event(enable_timing=True) for _ in range(k)] for _ in range(passes)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in range(passes):
        for j in range(k):
            starts[p][j].record()
            bfs_run(ws_h, int(sources[j]), level, parent)
            ends[p][j].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    ws.sync()
    ms = np.array([[a.elapsed_time(b) for a, b in zip(sa, se)] for sa, se in zip(starts, ends)])
    return ms, wall, bfs_kernel_times(ws_h)


def hm_gteps(ms, mc_half):
    """Harmonic mean over sources of GTEPS, each source at its median time over the passes."""
    ms = np.atleast_2d(ms)
    return hmean([mc_half[j] / (np.median(ms[:, j]) * 1e-3) / 1e9 for j in range(ms.shape[1])])


def host_info() -> dict:
    """The host the CPU baseline ran on: logical CPUs, the process's CPU share and the model."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    try:
        share = len(os.sched_getaffinity(0))
    except Exception:
        share = None
    return {"nproc": os.cpu_count(), "cpus_allowed": share, "lscpu_model": model}


def cpu_baseline(g, sources, threads: int, keep: bool = False):
    """The oracle (plain sequential BFS + parent pass) on `threads` host threads, one source
    each.  With keep, also returns each source's (level, parent) for the parity check."""
    import oracle
    oracle.build(force=False)
    res = [None] * threads
    outs = [None] * threads

    def work(i):
        s = int(sources[i % len(sources)])
        lv, par, tb, tp = oracle.timed_bfs(g.offsets, g.cols, s)
        mc = int(np.diff(g.offsets.astype(np.int64))[lv >= 0].sum())
        res[i] = (mc // 2, tb, tp)
        if keep:
            outs[i] = (s, lv, par)

    t0 = time.perf_counter()
    th = [threading.Thread(target=work, args=(i,)) for i in range(threads)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    wall = time.perf_counter() - t0
    edges = sum(r[0] for r in res)
    single = hmean([r[0] / (r[1] + r[2]) / 1e9 for r in res])
    host = host_info()
    out = {
        "value": round(edges / wall / 1e9, 5),
        "unit": "GTEPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{threads} of the workload's sources, one per host thread, search + parent pass each "
                  f"({wall:.1f} s wall); the thread count is the process's CPU share capped at 16",
        "host": host,
        "single_core_gteps_hmean": round(single, 5),
        "search_s_mean": round(float(np.mean([r[1] for r in res])), 3),
        "parent_s_mean": round(float(np.mean([r[2] for r in res])), 3),
    }
    return (out, outs) if keep else out


def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def short_name(name: str, width: int = 72) -> str:
    name = name.replace("s3bfs::", "").replace("(anonymous namespace)::", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def rocpd_summary(paths):
    """Per-kernel summary of rocprofv3 databases (kernel trace and/or counters), as text."""
    import sqlite3
    for path in paths:
        con = sqlite3.connect(path)
        print(f"# {path}")
        tabs = {r[0] for r in con.execute("select name from sqlite_master where type in ('table','view')")}
        if "top_kernels" in tabs:
            rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels "
                               "order by total_duration desc limit 10").fetchall()
            if rows:
                print("kernel | calls | total_us | avg_us | percent")
                for r in rows:
                    print(f"{short_name(r[0])} | {r[1]} | {r[2]:.1f} | {r[3]:.1f} | {r[4]:.2f}")
        if "counters_collection" in tabs:
            rows = con.execute("select kernel_name, counter_name, count(*), avg(value), min(value), max(value) "
                               "from counters_collection group by kernel_name, counter_name "
                               "order by avg(value) desc limit 12").fetchall()
            if rows:
                print("kernel | counter | dispatches | avg | min | max")
                for r in rows:
                    print(f"{short_name(r[0])} | {r[1]} | {r[2]} | {r[3]:.1f} | {r[4]:.1f} | {r[5]:.1f}")


def rocpd_dispatches(kernel: str, skip: int, take: int, path: str):
    """Durations of dispatches [skip, skip + take) of one kernel, in start order, from a
    rocprofv3 kernel-trace database (e.g. only the timed launches of the headline section)."""
    import sqlite3
    con = sqlite3.connect(path)
    rows = con.execute("select duration from kernels where name like ? order by start", (f"%{kernel}%",)).fetchall()
    d = np.array([r[0] for r in rows], dtype=np.float64)[skip: skip + take] / 1e6
    print(json.dumps({"kernel": kernel, "database": path, "dispatches_total": len(rows), "skip": skip,
                      "taken": int(d.size), "mean_ms": round(float(d.mean()), 4) if d.size else None,
                      "median_ms": round(float(np.median(d)), 4) if d.size else None,
                      "min_ms": round(float(d.min()), 4) if d.size else None,
                      "max_ms": round(float(d.max()), 4) if d.size else None}))


def traffic_from(paths, workload: str = "rmat24", kernel: str = "k_persistent<false>", out_dir: str = PROFILE_DIR):
    """Writes the HBM traffic per launch of the search kernel from four rocprofv3 counter
    databases (FETCH_SIZE and WRITE_SIZE of the bench run, then of the 1 GiB copy run), scaled
    by what the counters read for the copy, with the hash of the kernel source it belongs to."""
    import sqlite3

    def avg(path, counter, pattern):
        con = sqlite3.connect(path)
        r = con.execute("select avg(value), count(*) from counters_collection where counter_name = ? and "
                        "kernel_name like ?", (counter, pattern)).fetchone()
        return float(r[0] or 0.0), int(r[1])

    fetch_db, write_db, cfetch_db, cwrite_db = paths
    kpat = f"%{kernel}%"
    fetch, nd = avg(fetch_db, "FETCH_SIZE", kpat)
    write, nw = avg(write_db, "WRITE_SIZE", kpat)
    if nd == 0 or nw == 0:
        sys.exit(f"no dispatch of {kernel} in the counter databases")
    copy_bytes = 1 << 30
    cf, _ = avg(cfetch_db, "FETCH_SIZE", "%copyBuffer%")
    cw, _ = avg(cwrite_db, "WRITE_SIZE", "%copyBuffer%")
    ff = copy_bytes / (cf * 1024) if cf else float("nan")
    wf = copy_bytes / (cw * 1024) if cw else float("nan")
    out = {"kernel": kernel, "workload": f"{workload} (R-MAT scale 24, EF 16, 64 seeded sources cycled)",
           "kernel_source_sha256_16": kernel_source_hash(), "dispatches": nd,
           "fetch_kib_per_dispatch": round(fetch, 1), "write_kib_per_dispatch": round(write, 1),
           "copy_calibration": {"bytes": copy_bytes, "fetch_kib": round(cf, 1), "write_kib": round(cw, 1),
                                "fetch_factor": round(ff, 4), "write_factor": round(wf, 4)},
           "hbm_fetch_bytes_per_launch": int(fetch * 1024 * ff), "hbm_write_bytes_per_launch": int(write * 1024 * wf)}
    out["hbm_bytes_per_launch"] = out["hbm_fetch_bytes_per_launch"] + out["hbm_write_bytes_per_launch"]
    path = os.path.join(out_dir, f"traffic_persistent_{workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))
    return out


def counter_summary(kernel: str, paths):
    """Per-dispatch averages of the counters collected for `kernel` (a substring of its name)."""
    import sqlite3
    out = {"kernel": kernel}
    for path in paths:
        con = sqlite3.connect(path)
        for name, val, cnt in con.execute("select counter_name, avg(value), count(*) from counters_collection "
                                          "where kernel_name like ? group by counter_name", (f"%{kernel}%",)):
            out[name] = {"avg_per_dispatch": round(float(val), 1), "dispatches": int(cnt)}
    print(json.dumps(out))
    return out


def ws_options(pairs):
    """NAME=VALUE pairs of --ws-opt as Workspace keyword options."""
    out = {}
    for pair in pairs:
        name, _, value = pair.partition("=")
        out[name.strip()] = int(value)
    return out


def profile_c4(args):
    """The batched workload alone, for counter runs: R-MAT scale 22, 256 sources, the tuned
    launch shape from the package's tuning cache, `--steps` batches."""
    import torch

    from graphgen import workloads as W
    from paper_2209_08764_amd import Graph, Workspace, _lib
    _lib.load()
    g, srcs = W.c4_rmat22()
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G, max_sources=256)
    tune = ws.autotune(srcs, batch=True, cache=TUNE_CACHE)
    out = torch.empty(g.n * 256, dtype=torch.uint8, device="cuda")
    for _ in range(args.steps):
        ws.run_batch(srcs, out)
        ws.sync()
    print(json.dumps({"profile_c4": "rmat22 x 256 sources", "batches": args.steps,
                      "tuned": {k: tune.get(k) for k in ("batch_grain", "batch_tile", "batch_pull", "batch_levels",
                                                         "cached")}}), flush=True)


def calib_copy(args):
    """A plain device copy of known size: the reference for scaling rocprofv3's HBM counters."""
    import torch
    nbytes = 1 << 30
    x = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(4):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes": nbytes, "launches": 4}), flush=True)


def level_record(ws, small_edges: int = 16384, small_n: int = 4096):
    """Per-level (n_l, e_l, expand us, compact us, group level?) of the workspace's last run,
    from the level statistics and the device timestamps (a group level's compact us is its
    barrier)."""
    n_l, e_l = ws.level_stats()
    ex_us, co_us = ws.level_times()
    k = min(len(n_l), len(ex_us))
    return [[int(n_l[i]), int(e_l[i]), round(float(ex_us[i]), 2), round(float(co_us[i]), 2),
             bool(n_l[i] <= small_n and e_l[i] <= small_edges)] for i in range(k)]


def bench_c1(torch, W, Graph, Workspace):
    """R-MAT scale 16, one seeded source: microseconds per search."""
    g, srcs = W.c1_rmat16()
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G, profile=1)
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty_like(lv)
    s = int(srcs[0])
    ws.run(s, lv, pa)
    st = ws.stats()
    mc_half = st["edges"] / 2
    per_level = level_record(ws)
    ms, _, kms = time_passes(ws, lv, pa, [s], 200, torch)
    t = float(np.median(ms))
    return {"workload": "rmat16 (scale 16, EF 16), 1 source", "us_per_search": round(t * 1e3, 1),
            "kernel_us": round(float(np.median(kms)) * 1e3, 1), "gteps": round(mc_half / (t * 1e-3) / 1e9, 3),
            "levels": st["levels"], "small_levels": st["small_levels"], "grid": st["grid"],
            "per_level_nl_el_expand_us_compact_us_group": per_level}


def bench_c2(torch, W, Graph, Workspace):
    """4096 x 4096 grid from corner 0: a high-diameter search (8191 levels)."""
    g, srcs = W.c2_grid4096()
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G, profile=1)
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty_like(lv)
    ws.run(0, lv, pa)
    st = ws.stats()
    rec = level_record(ws)
    ms, _, kms = time_passes(ws, lv, pa, [0], 3, torch)
    t = float(np.median(ms))
    # split ablation: share start points by binary search instead of the scatter
    from paper_2209_08764_amd import BFS_OPT_SPLIT
    ws.set(BFS_OPT_SPLIT, 1)
    sm, _, _ = time_passes(ws, lv, pa, [0], 1, torch)
    ws.set(BFS_OPT_SPLIT, 0)
    t_search = float(np.median(sm))
    ws.run(0, lv, pa)
    W_ = 4096
    r, c = np.divmod(np.arange(g.n, dtype=np.int64), W_)
    closed_l = bool(np.array_equal(lv.cpu().numpy(), r + c))
    want_p = np.where(r > 0, (r - 1) * W_ + c, c - 1)
    want_p[0] = 0
    closed_p = bool(np.array_equal(pa.cpu().numpy(), want_p))
    one = [x for x in rec if x[4]]
    grid_lv = [x for x in rec if not x[4]]

    def us(rows):
        return round(float(np.mean([x[2] + x[3] for x in rows])), 2) if rows else None

    return {"workload": "grid 4096x4096 from vertex 0", "ms_per_search": round(t, 2),
            "kernel_ms": round(float(np.median(kms)), 2),
            "us_per_level": round(t * 1e3 / st["levels"], 2), "levels": st["levels"],
            "split_search_ms_per_search": round(t_search, 2),
            "small_levels": st["small_levels"], "gteps": round(st["edges"] / 2 / (t * 1e-3) / 1e9, 3),
            "closed_form_levels_ok": closed_l, "closed_form_parents_ok": closed_p,
            "us_per_level_group": us(one), "levels_group": len(one),
            "us_per_level_grid": us(grid_lv), "levels_grid": len(grid_lv),
            "per_level_sample_nl_el_expand_us_compact_us_group": rec[:4] + rec[500:504] + rec[1020:1028] +
            rec[2040:2052] + rec[4090:4100]}


class EnergyMeter:
    """GPU energy from amd-smi's accumulator (it advances about once a second): a sampling
    thread records each update, and the average power of a window is the energy between the
    first and last updates inside it over their time difference."""

    def __init__(self):
        import amdsmi
        self.smi = amdsmi
        amdsmi.amdsmi_init()
        self.h = amdsmi.amdsmi_get_processor_handles()[0]
        self.samples = []
        self.stop = threading.Event()
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def _run(self):
        last = None
        while not self.stop.is_set():
            e = self.smi.amdsmi_get_energy_count(self.h)
            key = (e["timestamp"], e["energy_accumulator"])
            if key != last:
                self.samples.append((time.perf_counter(), e["timestamp"], e["energy_accumulator"],
                                     e["counter_resolution"]))
                last = key
            time.sleep(0.02)

    def power(self, t0: float, t1: float):
        """Average watts between the first and last accumulator updates seen in [t0, t1]."""
        inside = [x for x in self.samples if t0 <= x[0] <= t1]
        if len(inside) < 2:
            return None
        a, b = inside[0], inside[-1]
        dt = (b[1] - a[1]) * 1e-9
        return (b[2] - a[2]) * b[3] * 1e-6 / dt if dt > 0 else None

    def close(self):
        self.stop.set()
        self.thread.join()
        self.smi.amdsmi_shut_down()


def energy_compare(torch, Graph, Workspace, graphs, seconds: float = 4.0) -> dict:
    """The paper's work-sensitivity claim on this GPU: energy per search of the work-sized level
    loop (BFS_MODE_AUTO: P_l = min(P, W_l) workgroups, group levels) against the
    work-insensitive variant (every workgroup active at every level), plus idle power."""
    from paper_2209_08764_amd import BFS_MODE_AUTO, BFS_MODE_INSENSITIVE
    try:
        meter = EnergyMeter()
    except Exception as ex:  # amd-smi missing or counters not readable
        return {"skipped": f"energy counters unavailable: {ex!r}"}
    out = {"method": "amd-smi energy accumulator (about 1 s updates), average power over a "
                     f"{seconds:.0f} s run of back-to-back searches x time per search"}
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        time.sleep(2.5)
        idle = meter.power(t0, time.perf_counter())
        out["idle_w"] = round(idle, 1) if idle else None
        for name, (G, sources) in graphs.items():
            n = G.n
            lv = torch.empty(n, dtype=torch.int32, device="cuda")
            pa = torch.empty_like(lv)
            for mode_name, mode in (("work_sensitive", BFS_MODE_AUTO), ("work_insensitive", BFS_MODE_INSENSITIVE)):
                ws = Workspace(G, mode=mode)
                ws.run(int(sources[0]), lv, pa)
                torch.cuda.synchronize()
                k = 0
                t0 = time.perf_counter()
                while time.perf_counter() - t0 < seconds or k < 2:
                    ws.run(int(sources[k % len(sources)]), lv, pa)
                    k += 1
                    if k % 4 == 0:
                        torch.cuda.synchronize()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                w = meter.power(t0, t1)
                ms = (t1 - t0) * 1e3 / k
                rec = {"ms_per_search": round(ms, 3), "avg_w": round(w, 1) if w else None,
                       "j_per_search": round(w * ms * 1e-3, 4) if w else None,
                       "dynamic_j_per_search": round((w - idle) * ms * 1e-3, 4) if (w and idle) else None}
                out[f"{name}_{mode_name}"] = rec
                ws.free()
            del lv, pa
    finally:
        meter.close()
    return out


TUNE_CACHE = os.path.join(ROOT, "paper_2209_08764_amd", "tuning_cache.json")


def bench_c4(torch, W, Graph, Workspace, g=None, srcs=None):
    """R-MAT scale 22, 256 sources in one batched run; versus single-source and plain runs,
    with a parity check of the whole batch against the oracle."""
    import concurrent.futures

    import oracle
    from paper_2209_08764_amd import BFS_MODE_PLAIN, BFS_OPT_MODE
    if g is None:
        g, srcs = W.c4_rmat22()
    G = Graph(g.offsets, g.cols)
    ws = Workspace(G, max_sources=256, profile=1)
    out = torch.empty(g.n * 256, dtype=torch.uint8, device="cuda")

    def timed_batches(reps=5):
        ws.run_batch(srcs, out)
        ws.sync()
        ws.kernel_times()
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ws.run_batch(srcs, out)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(times)), ws.kernel_times()

    t_default, _ = timed_batches()
    # the autotuner's launch shape for this graph and batch size, stored in the package's cache
    tune = ws.autotune(srcs, batch=True, cache=TUNE_CACHE)
    tb, kt = timed_batches()
    lev = out.view(g.n, 256)
    deg = torch.from_numpy(np.diff(g.offsets.astype(np.int64))).cuda()
    edges = float(sum(int(deg[lev[:, j] != 255].sum()) for j in range(256))) / 2
    n_l, e_l = ws.level_stats()
    # parity of the timed batch: the oracle's 256 searches on host threads, 16 sources each
    got = lev.cpu().numpy()
    blocks = [srcs[i:i + 16] for i in range(0, 256, 16)]
    with concurrent.futures.ThreadPoolExecutor(max_workers=host_cores()) as pool:
        parts = list(pool.map(lambda b: oracle.bfs_batch_u8(g.offsets, g.cols, b)[0], blocks))
    parity = bool(np.array_equal(got, np.concatenate(parts, axis=1)))
    del got, parts
    # 16 of the sources one at a time (single-source path), and the plain kernel on 4
    ss = Workspace(G, profile=1)
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty_like(lv)
    sm, _, _ = time_passes(ss, lv, pa, srcs[:16], 1, torch)
    single_ms = float(np.mean(sm))
    ss.set(BFS_OPT_MODE, BFS_MODE_PLAIN)
    pm, _, _ = time_passes(ss, lv, pa, srcs[:4], 1, torch)
    plain_ms = float(np.mean(pm))
    gteps = edges / (tb * 1e-3) / 1e9
    # algorithmic bytes of one batch: the uint8 output, each active row's columns, 40 B of
    # offsets and frontier mask per active vertex, 96 B of mask updates per newly reached vertex
    a_sum = float(np.sum(n_l))
    b_b = g.n * 256 + 4.0 * float(np.sum(e_l)) + 40.0 * a_sum + 96.0 * a_sum
    return {"workload": "rmat22 (scale 22, EF 16), 256 sources in one batched run",
            "ms_per_batch": round(tb, 3), "ms_per_batch_untuned": round(t_default, 3),
            "tuned": {k: tune.get(k) for k in ("batch_grain", "batch_tile", "batch_pull", "batch_levels", "trials",
                                                "cached")},
            "loop_ms": round(float(np.median(kt)), 3),
            "algorithmic_bytes": int(b_b), "hbm_frac_algorithmic": round(b_b / (tb * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "gteps_aggregate": round(gteps, 1), "levels": len(n_l),
            "active_per_level": n_l.tolist(), "active_edges_per_level": e_l.tolist(),
            "parity_256_sources_bit_exact": parity,
            "single_source_ms_mean": round(single_ms, 3),
            "speedup_vs_256_single_source": round(256 * single_ms / tb, 2),
            "plain_ms_mean": round(plain_ms, 2), "speedup_vs_256_plain": round(256 * plain_ms / tb, 1)}


class BusyMeter:
    """GPU activity (amd-smi's gfx activity percentage), sampled every 50 ms by a thread."""

    def __init__(self):
        import amdsmi
        self.smi = amdsmi
        amdsmi.amdsmi_init()
        self.h = amdsmi.amdsmi_get_processor_handles()[0]
        self.samples = []
        self.stop = threading.Event()
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def _run(self):
        while not self.stop.is_set():
            try:
                a = self.smi.amdsmi_get_gpu_activity(self.h)
                self.samples.append((time.perf_counter(), float(a["gfx_activity"])))
            except Exception:
                pass
            time.sleep(0.05)

    def mean(self, t0, t1):
        xs = [v for t, v in self.samples if t0 <= t <= t1]
        return float(np.mean(xs)) if xs else None

    def close(self):
        self.stop.set()
        self.thread.join()
        self.smi.amdsmi_shut_down()


def inflight_fraction(queries) -> float:
    """Fraction of the measured span during which at least one query was on the device."""
    iv = sorted((q.admitted, q.finished) for q in queries if q.admitted is not None)
    busy, cur0, cur1 = 0.0, None, None
    for a, b in iv:
        if cur1 is None or a > cur1:
            if cur1 is not None:
                busy += cur1 - cur0
            cur0, cur1 = a, b
        else:
            cur1 = max(cur1, b)
    if cur1 is not None:
        busy += cur1 - cur0
    span = max(q.finished for q in queries) - min(q.arrival for q in queries)
    return busy / span if span > 0 else 0.0


def bench_c5(torch, W, count: int, rmat22=None, warmup: int = 500):
    """Serving: 8 resident graphs, Poisson queries at the rate fixed in the workload recipe
    (0.7 x the closed-loop rate measured once), 2 GB admission budget."""
    from paper_2209_08764_amd.serve import GpuExecutor, Scheduler, latency_summary, poisson_queries
    graphs = W.c5_graphs() if rmat22 is None else W.c5_graphs_with(rmat22)
    ex = GpuExecutor(graphs, max_inflight=4)
    noniso = {k: np.flatnonzero(np.diff(g.offsets)) for k, g in graphs.items()}
    budget = W.C5_BUDGET_BYTES
    # answers are counted and dropped as they complete (10 000 level arrays would hold ~100 GB)
    sch = Scheduler(ex, budget_bytes=budget, max_inflight=4, keep_results=False)
    # closed loop (all queries at t = 0): the saturated rate, reported beside the frozen one
    closed = poisson_queries(graphs, noniso, rate=0, count=min(2000, count), seed=6)
    sch.run(closed)
    sat = latency_summary(closed)["qps"]
    rate = W.C5_RATE_QPS
    warm = poisson_queries(graphs, noniso, rate=rate, count=warmup, seed=5)
    sch.run(warm)
    qs = poisson_queries(graphs, noniso, rate=rate, count=count, seed=7)
    try:
        meter = BusyMeter()
    except Exception:
        meter = None
    t0 = time.perf_counter()
    sch.run(qs)
    t1 = time.perf_counter()
    busy = meter.mean(t0, t1) if meter else None
    if meter:
        meter.close()
    ok = [q for q in qs if q.error is None]
    summ = latency_summary(ok)
    sch.close()
    return {"workload": "8 resident graphs (rmat18/20/22/23, G(2^20, 8), grids 1024^2 and 2048^2, "
                        "power-law forest 2^20), Poisson arrivals",
            "rate_qps": rate, "rate_rule": "0.7 x the closed-loop rate, measured once and fixed in the recipe",
            "closed_loop_qps_this_run": round(sat, 1), "warmup_queries": warmup, "queries": count,
            "failed": len(qs) - len(ok),
            "p50_ms": round(summ["p50_ms"], 3), "p99_ms": round(summ["p99_ms"], 3),
            "mean_ms": round(summ["mean_ms"], 3), "qps": round(summ["qps"], 1),
            "batched_fraction": round(summ["batched_fraction"], 3), "budget_bytes": budget,
            "gpu_busy_pct_amdsmi": round(busy, 1) if busy is not None else None,
            "inflight_pct": round(100 * inflight_fraction(ok), 1), "scheduler": dict(sch.stats)}


def bench_multiroot(torch, Graph, Workspace, count: int = 1024):
    """Many small graphs: a disjoint union searched from one root per part in one launch
    (bfs_run_multiroot), against one search per part on its own resident graph."""
    import graphgen as gg
    import oracle
    parts = []
    for i in range(count):
        kind = i % 4
        if kind == 0:
            parts.append(gg.rmat(10, seed=7000 + i))
        elif kind == 1:
            parts.append(gg.grid(16 + i % 17, 24))
        elif kind == 2:
            parts.append(gg.powerlaw_forest(1500, nroots=1, seed=7000 + i))
        else:
            parts.append(gg.erdos_renyi(1000, 6.0, seed=7000 + i))
    u, base = gg.disjoint_union(parts)
    roots = np.array([int(base[i]) + int(gg.pick_sources(p, 1, seed=i)[0]) for i, p in enumerate(parts)], np.int32)
    G = Graph(u.offsets, u.cols)
    ws = Workspace(G, profile=1)
    lv = torch.empty(u.n, dtype=torch.int32, device="cuda")
    pa = torch.empty_like(lv)
    ws.run_multiroot(roots, lv, pa)
    ws.sync()
    want_l, want_p = oracle.bfs(u.offsets, u.cols, roots)
    parity = bool(np.array_equal(lv.cpu().numpy(), want_l) and np.array_equal(pa.cpu().numpy(), want_p))
    times = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ws.run_multiroot(roots, lv, pa)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    t_union = float(np.median(times))
    # one search per part, each part resident on its own, back to back on one stream
    sep = [(Graph(p.offsets, p.cols), int(r - b)) for p, r, b in zip(parts, roots, base)]
    wss = [(Workspace(Gp), s, torch.empty(Gp.n, dtype=torch.int32, device="cuda"),
            torch.empty(Gp.n, dtype=torch.int32, device="cuda")) for Gp, s in sep]
    for w, s, l, q in wss[:8]:
        w.run(s, l, q)
    torch.cuda.synchronize()
    sp = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for w, s, l, q in wss:
            w.run(s, l, q)
        torch.cuda.synchronize()
        sp.append((time.perf_counter() - t0) * 1e3)
    t_sep = float(np.median(sp))
    for w, _, _, _ in wss:
        w.free()
    for Gp, _ in sep:
        Gp.free()
    mc = int(np.diff(u.offsets.astype(np.int64))[want_l >= 0].sum()) // 2
    return {"workload": f"disjoint union of {count} small graphs (R-MAT 10, grids, forests, G(1000, 6)), "
                        "one root each", "n": u.n, "m": u.m, "ms_one_launch": round(t_union, 3),
            "ms_separate_searches": round(t_sep, 3), "speedup": round(t_sep / t_union, 2),
            "gteps_one_launch": round(mc / (t_union * 1e-3) / 1e9, 3), "parity_bit_exact": parity}


def probe_ceiling(torch, n: int, count: int = 1 << 28, reps: int = 5) -> dict:
    """Random-probe rate of the device for the expansion's two probe patterns: a bit of an
    n-bit bitmap (n / 8 bytes, L2-resident) and an entry of an n-entry int32 array (4n bytes)."""
    from paper_2209_08764_amd import bfs_probe_rate_kernel
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    idx = torch.randint(0, n, (count,), dtype=torch.int32, device="cuda", generator=gen)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = {}
    for name, words, shift in [("bitmap", (n + 31) // 32, 5), ("level_array", n, 0)]:
        table = torch.zeros(words, dtype=torch.int32, device="cuda")
        bfs_probe_rate_kernel(idx, table, shift, sink)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            bfs_probe_rate_kernel(idx, table, shift, sink)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[f"{name}_{words * 4 // 1024}KiB_gprobes_per_s"] = round(count / (ms * 1e-3) / 1e9, 1)
        del table
    del idx
    torch.cuda.empty_cache()
    return out


def run_only(args):
    """Some of the other workloads alone, for quick measurements (no headline line)."""
    import torch

    from graphgen import workloads as W
    from paper_2209_08764_amd import Graph, Workspace, _lib
    _lib.load()
    torch.cuda.set_device(0)
    out = {}
    for name in [x.strip() for x in args.only.split(",") if x.strip()]:
        log(name)
        if name == "c1":
            out[name] = bench_c1(torch, W, Graph, Workspace)
        elif name == "c2":
            out[name] = bench_c2(torch, W, Graph, Workspace)
        elif name == "c4":
            out[name] = bench_c4(torch, W, Graph, Workspace)
        elif name == "multiroot":
            out[name] = bench_multiroot(torch, Graph, Workspace)
        elif name == "c5":
            out[name] = bench_c5(torch, W, args.serve_queries)
        else:
            sys.exit(f"unknown workload {name}")
        log(f"  {dict((k, v) for k, v in out[name].items() if not k.startswith('per_level'))}")
        torch.cuda.empty_cache()
    print(json.dumps({"only": out}), flush=True)


def run(args):
    import torch

    import graphgen as gg
    from graphgen import workloads as W
    from paper_2209_08764_amd import (BFS_MODE_AUTO, BFS_MODE_DIRECTION, BFS_MODE_INSENSITIVE, BFS_MODE_LEVEL,
                                      BFS_MODE_PLAIN, BFS_OPT_DENSE_EDGES, BFS_OPT_MODE, BFS_OPT_PROFILE, BFS_OPT_SPLIT,
                                      Graph, Workspace, _lib)

    _lib.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    log(f"generating R-MAT scale {args.scale} ({gg.num_threads()} host threads)")
    t = time.perf_counter()
    g, sources = W.c3_rmat24(scale=args.scale, nsrc=64)
    log(f"  n={g.n} m={g.m} in {time.perf_counter() - t:.1f} s")
    G = Graph(g.offsets, g.cols)
    ablation = ws_options(args.ws_opt)
    ws = Workspace(G, profile=1, **ablation)
    n = g.n
    level = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")

    # per-source component sizes and per-level records from one untimed pass (also a warm-up)
    mc_half, nc, per_level = [], [], []
    for j, s in enumerate(sources):
        ws.run(int(s), level, parent)
        st = ws.stats()
        if st["status"] != 0:
            raise RuntimeError(f"device status {st['status']} on source {s}")
        mc_half.append(st["edges"] / 2)
        nc.append(st["reached"])
        levels_used = st["levels"]
        if j < 4:
            per_level.append({"source": int(s), "grid": st["grid"], "levels": level_record(ws)})
    for _ in range(args.warmup):
        for s in sources:
            ws.run(int(s), level, parent)
    ws.sync()
    log(f"timing {args.steps} passes over the {len(sources)} sources")
    step_ms, wall_ms, kms = time_passes(ws, level, parent, sources, args.steps, torch)
    value = hm_gteps(step_ms, mc_half)
    # roofline of the persistent kernel: every source once per pass, so the mean over sources
    kb = float(np.mean([algorithmic_bytes(n, nc[j], int(2 * mc_half[j]))[1] for j in range(len(sources))]))
    kt = float(np.mean(kms)) if len(kms) else float("nan")
    achieved = kb / (kt * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if ablation else stored_traffic("rmat24"),
                "traffic_source": "stored rocprofv3 FETCH_SIZE + WRITE_SIZE runs of this kernel code "
                                  "(profiles/traffic_persistent_rmat24.json, keyed by source hash; "
                                  "null once the code changes)",
                "kernel": "k_persistent<false>", "kernel_ms_mean": round(kt, 4), "launches": int(len(kms)),
                "algorithmic_bytes_per_launch": int(kb), "target_frac": 0.40}
    log(f"single-source: {value:.2f} GTEPS hm, {np.mean(step_ms):.3f} ms/search, kernel {kt:.3f} ms, "
        f"{achieved:.0f} GB/s algorithmic")

    extras = {"levels": levels_used, "n": n, "m": g.m, "search_ms_median": round(float(np.median(step_ms)), 4),
              "searches_timed": int(step_ms.size), "c3_per_level_first_4_sources": per_level}
    # the secondary ceiling: every scanned edge probes the visited bitmap at a random word
    ceil = probe_ceiling(torch, n)
    probes = float(np.mean([2 * x for x in mc_half])) / (kt * 1e-3) / 1e9
    bkey = next(k for k in ceil if k.startswith("bitmap"))
    extras["probe_ceiling"] = ceil
    extras["probe_rate_gprobes_per_s"] = round(probes, 1)
    extras["probe_ceiling_frac"] = round(probes / ceil[bkey], 4)
    log(f"probe ceiling {ceil}; the search probes at {probes:.1f} G/s")
    if not args.quick:
        ws.set(BFS_OPT_PROFILE, 0)
        for name, mode, nsrc in [("plain", BFS_MODE_PLAIN, 8), ("level", BFS_MODE_LEVEL, 8),
                                 ("insensitive", BFS_MODE_INSENSITIVE, 16), ("direction", BFS_MODE_DIRECTION, 64)]:
            ws.set(BFS_OPT_MODE, mode)
            sub = sources[:nsrc]
            for s in sub[:2]:
                ws.run(int(s), level, parent)
            ws.sync()
            sm, _, _ = time_passes(ws, level, parent, sub, 1, torch)
            extras[f"{name}_gteps_hm"] = round(hm_gteps(sm, mc_half[:nsrc]), 3)
            extras[f"{name}_ms_median"] = round(float(np.median(sm)), 3)
            log(f"{name}: {extras[f'{name}_gteps_hm']} GTEPS")
        ws.set(BFS_OPT_MODE, BFS_MODE_AUTO)
        extras["speedup_vs_plain"] = round(value / extras["plain_gteps_hm"], 2)
        # split ablation: share start points by binary search instead of the scatter
        ws.set(BFS_OPT_SPLIT, 1)
        sub = sources[:16]
        for s in sub[:2]:
            ws.run(int(s), level, parent)
        ws.sync()
        sm, _, _ = time_passes(ws, level, parent, sub, 1, torch)
        extras["split_search_gteps_hm"] = round(hm_gteps(sm, mc_half[:16]), 3)
        extras["split_search_ms_median"] = round(float(np.median(sm)), 3)
        extras["split_scatter_gteps_hm_same_sources"] = round(hm_gteps(step_ms[:, :16], mc_half[:16]), 3)
        ws.set(BFS_OPT_SPLIT, 0)
        log(f"split by binary search: {extras['split_search_gteps_hm']} GTEPS")
        # the paper's private queues and Owner test on every level (no dense levels), same launch
        dense_default = ws.tuning()["dense_edges"]
        ws.set(BFS_OPT_DENSE_EDGES, 0)
        for s in sub[:2]:
            ws.run(int(s), level, parent)
        ws.sync()
        sm, _, _ = time_passes(ws, level, parent, sub, 1, torch)
        extras["queues_every_level_gteps_hm"] = round(hm_gteps(sm, mc_half[:16]), 3)
        extras["queues_every_level_ms_median"] = round(float(np.median(sm)), 3)
        ws.set(BFS_OPT_DENSE_EDGES, dense_default)   # the default threshold again
        log(f"private queues and Owner test on every level: {extras['queues_every_level_gteps_hm']} GTEPS")
        # energy: work-sized against work-insensitive levels, on this graph and on the grid
        log("energy: work-sensitive vs work-insensitive (R-MAT 24, grid 4096^2)")
        gg2, _ = W.c2_grid4096()
        Ggrid = Graph(gg2.offsets, gg2.cols)
        extras["energy"] = energy_compare(torch, Graph, Workspace,
                                          {"rmat24": (G, sources), "grid4096": (Ggrid, [0])})
        Ggrid.free()
        del gg2
        log(f"  {extras['energy']}")
        # ablation: the same search without the hot-vertex filter (same resident CSR, borrowed)
        if G.aux_bytes:
            lean = Graph(G.offsets, G.cols, hot=False)
            wl = Workspace(lean)
            sub = sources[:16]
            for s in sub[:2]:
                wl.run(int(s), level, parent)
            wl.sync()
            sm, _, _ = time_passes(wl, level, parent, sub, 1, torch)
            extras["no_hot_filter_gteps_hm"] = round(hm_gteps(sm, mc_half[:16]), 3)
            extras["hot_filter_aux_bytes"] = G.aux_bytes
            log(f"without the hot-vertex filter: {extras['no_hot_filter_gteps_hm']} GTEPS")
            wl.free()
            lean.free()

    cpu = None
    if not args.no_cpu:
        threads = host_cores()
        log(f"CPU oracle baseline on {threads} host threads")
        cpu, outs = cpu_baseline(g, sources, threads, keep=True)
        log(f"  oracle {cpu['value']} GTEPS on {threads} threads ({cpu['host']})")
        # parity of the timed configuration on the sources the oracle just solved
        ok = 0
        for s, want_l, want_p in outs:
            ws.run(s, level, parent)
            ws.sync()
            ok += int(np.array_equal(level.cpu().numpy(), want_l) and np.array_equal(parent.cpu().numpy(), want_p))
        extras["parity_checked_sources"] = len(outs)
        extras["parity_bit_exact_sources"] = ok
        log(f"  parity: {ok} of {len(outs)} sources bit-exact (level and parent)")
        del outs
    ws.free()
    G.free()
    del level, parent, ws, G, g
    torch.cuda.empty_cache()

    if not args.quick:
        log("C1: R-MAT 16")
        extras["c1"] = bench_c1(torch, W, Graph, Workspace)
        log(f"  {extras['c1']}")
        log("C2: grid 4096x4096")
        extras["c2"] = bench_c2(torch, W, Graph, Workspace)
        log(f"  {dict((k, v) for k, v in extras['c2'].items() if not k.startswith('per_level'))}")
        torch.cuda.empty_cache()
        log("C4: R-MAT 22, 256 sources batched")
        g22, s22 = W.c4_rmat22()
        extras["c4"] = bench_c4(torch, W, Graph, Workspace, g22, s22)
        log(f"  {extras['c4']}")
        torch.cuda.empty_cache()
        log("many small graphs in one multi-root launch")
        extras["multiroot"] = bench_multiroot(torch, Graph, Workspace)
        log(f"  {extras['multiroot']}")
        torch.cuda.empty_cache()
        if args.serve_queries > 0:
            log(f"C5: serving, {args.serve_queries} queries")
            extras["c5"] = bench_c5(torch, W, args.serve_queries, rmat22=g22)
            log(f"  {extras['c5']}")

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_64src_single", "graph": "R-MAT", "scale": args.scale,
                   "edgefactor": 16, "abcd": [0.57, 0.19, 0.19, 0.05], "symmetrised": True, "permuted": True,
                   "sources": len(sources), "sources_timed_per_step": len(sources),
                   "step": "one pass over all sources, one search at a time", "mode": "auto",
                   "hot_vertex_filter": True, "gteps_edges": "undirected edges in the component",
                   **({"ablation_workspace_options": ablation} if ablation else {})},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed passes over the 64 sources")
    ap.add_argument("--warmup", type=int, default=1, help="untimed passes before them")
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--only", default="", help="comma-separated extras to run without the headline "
                                               "(c1, c2, c4, multiroot, c5); prints them and exits")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serve-queries", type=int, default=10000, help="queries in the serving run (0 skips it)")
    ap.add_argument("--calib-copy", action="store_true", help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--profile-c4", action="store_true", help="only run --steps batches of the batched workload "
                                                              "(counter runs)")
    ap.add_argument("--rocpd-summary", nargs="+", metavar="DB", help="summarise rocprofv3 result databases and exit")
    ap.add_argument("--rocpd-dispatches", nargs=4, metavar=("KERNEL", "SKIP", "TAKE", "DB"),
                    help="duration statistics of dispatches [SKIP, SKIP+TAKE) of KERNEL in start order, and exit")
    ap.add_argument("--ws-opt", action="append", default=[], metavar="NAME=VALUE",
                    help="workspace option of the headline run (an ablation: e.g. dense_edges=0); repeatable")
    ap.add_argument("--counter-summary", nargs="+", metavar=("KERNEL", "DB"),
                    help="per-dispatch averages of every counter of KERNEL in rocprofv3 counter databases, "
                         "and exit")
    ap.add_argument("--traffic-from", nargs=4, metavar="DB",
                    help="FETCH_SIZE and WRITE_SIZE databases of the bench run, then of --calib-copy: write the "
                         "search kernel's HBM traffic per launch to profiles/ and exit")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(args.traffic_from)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary[0], args.counter_summary[1:])
        return
    if args.rocpd_dispatches:
        k, skip, take, db = args.rocpd_dispatches
        rocpd_dispatches(k, int(skip), int(take), db)
        return
    if args.rocpd_summary:
        rocpd_summary(args.rocpd_summary)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the search runs on a single MI355X "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy(args)
        return
    if args.profile_c4:
        profile_c4(args)
        return
    if args.only:
        run_only(args)
        return
    run(args)


if __name__ == "__main__":
    main()
