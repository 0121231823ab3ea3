"""The oracle (oracle/oracle.c) and the input generators (graphgen/gen.c) built with
AddressSanitizer and UndefinedBehaviorSanitizer, exercised in a child process on the
CPU: every graph family, sources, single- and multi-root searches, parents and the
batched uint8 layout, on ordinary and degenerate inputs.  Any report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import graphgen as gg
import oracle
from oracle.brute import adjacency, floyd_warshall
graphs = [gg.rmat(11, seed=3), gg.rmat(8, seed=4, permute=False), gg.grid(37, 23), gg.grid(1, 500),
          gg.erdos_renyi(3000, 5.0, seed=2), gg.powerlaw_forest(4000, seed=5), gg.from_edges(1, []),
          gg.from_edges(7, [(0, 1), (1, 2), (4, 5)])]
u, base = gg.disjoint_union(graphs[:4])
graphs.append(u)
for g in graphs:
    srcs = gg.pick_sources(g, min(5, int((np.diff(g.offsets) > 0).sum())), seed=9) if g.m else np.array([0])
    for s in srcs:
        lv, par = oracle.bfs(g.offsets, g.cols, int(s))
        assert lv[s] == 0 and par[s] == s
    if g.m:
        lv, par = oracle.bfs(g.offsets, g.cols, srcs)
        out, ovf = oracle.bfs_batch_u8(g.offsets, g.cols, np.resize(srcs, 70))
        assert out.shape == (g.n, 70)
        t = oracle.timed_bfs(g.offsets, g.cols, int(srcs[0]))
        assert np.array_equal(t[0], oracle.bfs_levels(g.offsets, g.cols, int(srcs[0])))
small = gg.rmat(5, seed=1)
D = floyd_warshall(adjacency(small.n, small.offsets, small.cols))
for s in range(small.n):
    assert np.array_equal(oracle.bfs_levels(small.offsets, small.cols, s), D[s])
print("SANITIZED_RUN_OK")
"""


def _build(src, out, extra):
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-o", out, src] + extra
    subprocess.check_call(cmd)


def test_oracle_and_generators_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("libasan not available")
    olib = str(tmp_path / "liboracle_san.so")
    glib = str(tmp_path / "libgraphgen_san.so")
    _build(os.path.join(ROOT, "oracle", "oracle.c"), olib, [])
    _build(os.path.join(ROOT, "graphgen", "gen.c"), glib, ["-fopenmp", "-lm"])
    env = dict(os.environ, LD_PRELOAD=libasan, S3BFS_ORACLE_LIB=olib, S3BFS_GRAPHGEN_LIB=glib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=87", OMP_NUM_THREADS="4")
    res = subprocess.run([sys.executable, "-c", DRIVER, ROOT], env=env, capture_output=True, text=True,
                         timeout=600)
    report = res.stdout[-3000:] + res.stderr[-6000:]
    assert res.returncode == 0, report
    assert "SANITIZED_RUN_OK" in res.stdout, report
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, report
