"""The five benchmark workloads as seeded input recipes (input generation only).

C1 rmat16    R-MAT scale 16, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), one source
C2 grid4096  4096 x 4096 4-neighbour grid, source = corner vertex 0
C3 rmat24    R-MAT scale 24, edge factor 16, 64 sources run one at a time
C4 rmat22    R-MAT scale 22, edge factor 16, 256 sources in one batched launch
C5 serve8    eight resident graphs for the serving loop

Sources are drawn uniformly among vertices of degree >= 1 (distinct within
one workload).  All R-MAT graphs are symmetrised, deduplicated and
vertex-permuted.  The paper's own inputs (a Wikipedia graph, unnamed
real-world and synthetic graphs) are not available; these stand in.
"""
from __future__ import annotations

from . import erdos_renyi, grid, pick_sources, powerlaw_forest, rmat

# C5 serving: queries arrive at a fixed Poisson rate, 0.7 x the closed-loop (saturated) rate of
# the serving loop on one MI355X (417.3 queries/s, all queries queued at once, measured once with
# this graph set and scheduler), under a 2 GB admission budget for workspaces and outputs.
C5_RATE_QPS = 292.0
C5_BUDGET_BYTES = 2_000_000_000

SEEDS = {
    "rmat16": (1601, 1602),
    "rmat24": (2401, 2402),
    "rmat22": (2201, 2202),
    "rmat18": (1801, 1802),
    "rmat20": (2001, 2002),
    "rmat23": (2301, 2302),
    "er20": (3001, 3002),
    "forest20": (3101, 3102),
}


def c1_rmat16():
    g = rmat(16, 16, seed=SEEDS["rmat16"][0])
    return g, pick_sources(g, 1, seed=SEEDS["rmat16"][1])


def c2_grid4096(W: int = 4096):
    g = grid(W, W)
    import numpy as np
    return g, np.array([0], dtype=np.int32)


def c3_rmat24(scale: int = 24, nsrc: int = 64):
    g = rmat(scale, 16, seed=SEEDS["rmat24"][0])
    return g, pick_sources(g, nsrc, seed=SEEDS["rmat24"][1])


def c4_rmat22(scale: int = 22, nsrc: int = 256):
    g = rmat(scale, 16, seed=SEEDS["rmat22"][0])
    return g, pick_sources(g, nsrc, seed=SEEDS["rmat22"][1])


def c5_graphs_with(rmat22):
    """The serving set reusing an already generated R-MAT 22 (same seed as C4)."""
    return {
        "rmat18": rmat(18, 16, seed=SEEDS["rmat18"][0]),
        "rmat20": rmat(20, 16, seed=SEEDS["rmat20"][0]),
        "rmat22": rmat22,
        "rmat23": rmat(23, 16, seed=SEEDS["rmat23"][0]),
        "er20": erdos_renyi(1 << 20, 8.0, seed=SEEDS["er20"][0]),
        "grid1024": grid(1024, 1024),
        "grid2048": grid(2048, 2048),
        "forest20": powerlaw_forest(1 << 20, seed=SEEDS["forest20"][0]),
    }


def c5_graphs(small: bool = False):
    """The serving set: name -> graph.  small=True shrinks every graph (tests)."""
    if small:
        return {
            "rmat10": rmat(10, 16, seed=SEEDS["rmat18"][0]),
            "rmat11": rmat(11, 16, seed=SEEDS["rmat20"][0]),
            "rmat12": rmat(12, 16, seed=SEEDS["rmat22"][0]),
            "er12": erdos_renyi(1 << 12, 8.0, seed=SEEDS["er20"][0]),
            "grid64": grid(64, 64),
            "grid48": grid(48, 48),
            "forest12": powerlaw_forest(1 << 12, seed=SEEDS["forest20"][0]),
        }
    return {
        "rmat18": rmat(18, 16, seed=SEEDS["rmat18"][0]),
        "rmat20": rmat(20, 16, seed=SEEDS["rmat20"][0]),
        "rmat22": rmat(22, 16, seed=SEEDS["rmat22"][0]),
        "rmat23": rmat(23, 16, seed=SEEDS["rmat23"][0]),
        "er20": erdos_renyi(1 << 20, 8.0, seed=SEEDS["er20"][0]),
        "grid1024": grid(1024, 1024),
        "grid2048": grid(2048, 2048),
        "forest20": powerlaw_forest(1 << 20, seed=SEEDS["forest20"][0]),
    }
