"""GPU parity of the level-loop primitive (owner de-duplication + linearisation +
next-level degree prefix sum + share start points) against the oracle's
primitive-by-primitive step model (oracle/s3bfs_steps.py).

The survivors are a set (their order across queues is not part of the
result), so the test compares the survivor multiset exactly and checks that
the degree prefix sums and the share start points the GPU wrote are the ones
the step model's running totals and chunk starts give for the GPU's output
order.
"""
import numpy as np
import pytest

import graphgen as gg
from oracle import s3bfs_steps as st

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2209_08764_amd import bfs_prim_compact, bfs_prim_grain  # noqa: E402


def _case(g, ntiles, seed, fill):
    grain = bfs_prim_grain()
    rng = np.random.default_rng(seed)
    cnt = np.minimum(rng.integers(0, grain + 1, ntiles), int(fill * grain)).astype(np.int32)
    if ntiles:
        cnt[rng.integers(0, ntiles)] = grain            # one full queue
        cnt[rng.integers(0, ntiles)] = 0                # one empty queue
    cand = np.full(ntiles * grain, -7, np.int32)
    slots_of = {}
    for t in range(ntiles):
        vs = rng.integers(0, g.n, cnt[t]).astype(np.int32)
        cand[t * grain:t * grain + cnt[t]] = vs
        for i, v in enumerate(vs):
            slots_of.setdefault(int(v), []).append(t * grain + i)
    owner = np.full(g.n, -1, np.int32)
    for v, slots in slots_of.items():
        # the last writer wins: usually one of the slots that hold v, sometimes none of them
        owner[v] = slots[rng.integers(0, len(slots))] if rng.random() < 0.9 else -5
    return cnt, cand, owner


def _oracle(g, cnt, cand, owner):
    grain = bfs_prim_grain()
    Q = [list(cand[t * grain:t * grain + cnt[t]]) for t in range(len(cnt))]
    # Owner[v] holds a global slot here; queue i keeps v when that slot is one of its own entries
    keep = []
    for t, q in enumerate(Q):
        for i, v in enumerate(q):
            if owner[v] == t * grain + i:
                keep.append(int(v))
    deg = np.diff(g.offsets)
    frontier = [v for v in keep if deg[v] > 0]
    return sorted(frontier), len(frontier), int(sum(deg[v] for v in frontier))


@pytest.mark.parametrize("ntiles,seed,fill", [(1, 1, 1.0), (3, 2, 0.01), (37, 3, 1.0), (130, 4, 0.3),
                                              (700, 5, 0.05), (0, 6, 1.0)])
def test_prim_compact_matches_oracle_steps(ntiles, seed, fill):
    g = gg.rmat(12, seed=seed)
    grain = bfs_prim_grain()
    cnt, cand, owner = _case(g, ntiles, seed, fill)
    want_set, want_n, want_e = _oracle(g, cnt, cand, owner)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    offsets = dev(g.offsets)
    out_v = torch.full((g.n,), -3, dtype=torch.int32, device="cuda")
    out_rs = torch.full((g.n,), -3, dtype=torch.int32, device="cuda")
    out_ex = torch.full((g.n + 1,), -3, dtype=torch.int32, device="cuda")
    cap = (g.m + grain - 1) // grain + 2
    out_ts = torch.full((cap,), -3, dtype=torch.int32, device="cuda")
    totals = torch.zeros(2, dtype=torch.int32, device="cuda")
    bfs_prim_compact(offsets, dev(owner), dev(cand if cand.size else np.zeros(1, np.int32)),
                     dev(cnt if cnt.size else np.zeros(0, np.int32)), out_v, out_rs, out_ex, out_ts, totals)
    torch.cuda.synchronize()
    n_out, e_out = totals.cpu().tolist()
    assert (n_out, e_out) == (want_n, want_e)
    v = out_v.cpu().numpy()[:n_out]
    assert sorted(v.tolist()) == want_set
    np.testing.assert_array_equal(out_rs.cpu().numpy()[:n_out], g.offsets[v])
    # degree gather + prefix sum on the GPU's output order
    incl = st.running_totals(st.row_lengths(v.tolist(), g.offsets))
    ex = out_ex.cpu().numpy()[:n_out + 1]
    np.testing.assert_array_equal(ex, [0] + incl if n_out else [0])
    # chunk starts (Find-StartExpPoint) with the grain as chunk size
    if want_e:
        P = -(-want_e // grain)
        starts = st.chunk_starts(incl, want_e, P, size=grain)
        np.testing.assert_array_equal(out_ts.cpu().numpy()[:P], [j for (j, _) in starts])
