"""Input generators: structure and determinism (no GPU)."""
import numpy as np
import pytest

import graphgen as gg


def _check_csr(g):
    off, cols = g.offsets.astype(np.int64), g.cols.astype(np.int64)
    assert off[0] == 0 and off[-1] == g.m and (np.diff(off) >= 0).all()
    if g.m:
        assert cols.min() >= 0 and cols.max() < g.n
    src = np.repeat(np.arange(g.n), np.diff(off))
    assert not (src == cols).any(), "self-loop"
    same_row = src[1:] == src[:-1]
    assert (cols[1:][same_row] > cols[:-1][same_row]).all(), "unsorted or duplicate"
    fwd = np.sort(src * g.n + cols)
    bwd = np.sort(cols * g.n + src)
    assert np.array_equal(fwd, bwd), "not symmetric"


@pytest.mark.parametrize("make", [lambda: gg.rmat(10, seed=1), lambda: gg.rmat(12, 8, seed=2, permute=False),
                                  lambda: gg.grid(17, 5), lambda: gg.grid(1, 9), lambda: gg.grid(1, 1),
                                  lambda: gg.erdos_renyi(3000, 8, seed=3),
                                  lambda: gg.powerlaw_forest(4000, seed=4)])
def test_symmetric_sorted_dedup(make):
    _check_csr(make())


def test_determinism_and_seed_sensitivity():
    a, b, c = gg.rmat(11, seed=5), gg.rmat(11, seed=5), gg.rmat(11, seed=6)
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.cols, b.cols)
    assert not (np.array_equal(a.offsets, c.offsets) and np.array_equal(a.cols, c.cols))
    assert np.array_equal(gg.pick_sources(a, 7, seed=3), gg.pick_sources(b, 7, seed=3))


def test_grid_counts_and_forest_is_a_forest():
    g = gg.grid(4096 // 64, 4096 // 64)
    assert g.m == 2 * (2 * 64 * 63)
    f = gg.powerlaw_forest(1 << 12, nroots=64, seed=1)
    assert f.m == 2 * ((1 << 12) - 64)          # n - 64 distinct tree edges
    from oracle.certify import components
    assert len(np.unique(components(f.offsets, f.cols))) == 64


def test_rmat_shape_matches_recipe():
    g = gg.rmat(14, seed=1)
    deg = g.degrees()
    assert g.n == 1 << 14
    # symmetrised and deduplicated: close to but below 2 * EF * n entries
    assert 0.8 * 2 * 16 * g.n < g.m < 2 * 16 * g.n
    assert 0.15 < (deg == 0).mean() < 0.4         # R-MAT leaves many isolated vertices
    assert deg.max() > 50 * deg.mean()            # heavy tail


def test_sources_are_non_isolated_and_distinct():
    g = gg.rmat(10, seed=2)
    s = gg.pick_sources(g, 200, seed=9)
    assert len(set(s.tolist())) == 200 and (g.degrees()[s] > 0).all()
    with pytest.raises(ValueError):
        gg.pick_sources(gg.from_edges(4, [(0, 1)]), 3, distinct=True)


def test_disjoint_union():
    u, base = gg.disjoint_union([gg.grid(3, 2), gg.from_edges(3, [(0, 2)]), gg.grid(2, 2)])
    _check_csr(u)
    assert base.tolist() == [0, 6, 9] and u.n == 13
