"""Reference model of one level-synchronous search step, primitive by primitive
(test infrastructure only: used by tests/, never by the GPU library).

S3BFS (Figure 1 with the Algorithm and Analysis paragraphs) advances a
frontier in rounds.  Each round is built from a handful of data-parallel
primitives; this module gives each one as a small, slow, obviously correct
function of its own, and a driver that chains them.  Workers are simulated
one after another.  The functions are checked independently: the chunk
starts against numpy's searchsorted, the concatenation and ownership filter
against their set semantics, and the whole round loop against the plain
BFS oracle, with and without a model of racing workers.

The primitives, in the project's terms (the paper's names in brackets):

  row_lengths        degree of every frontier vertex        [degree gather]
  running_totals     inclusive prefix sums                   [Parallel-Prefix-Sum]
  chunk_starts       where each worker's equal chunk of the  [Find-StartExpPoint]
                     round's edges begins: entry and offset
  scan_chunks        each worker walks its chunk of edges    [EXPLORE-VERTEX]
                     and lists the unvisited targets it
                     claims
  keep_claimed       drop a listed vertex unless the list    [owner de-duplication]
                     holds its final claim
  concatenate        the lists, one after another, at the    [linearisation]
                     running totals of their lengths

Readings where the paper is silent (each also in the design notes):
  * EXPLORE-VERTEX has no body in the paper.  From the Algorithm paragraph:
    a worker that finds a target with no distance yet gives it the round's
    distance, records itself as the target's claimant and lists it; workers
    race, every racer writes the same distance, and the last claim stands.
  * Chunks are equal runs of ceil(edges / workers) consecutive edges (the
    paper asks for nearly equal shares), unless a fixed chunk size is given.
  * The scatter form of the chunk starts: the frontier entry covering edges
    [a, b) is where every chunk whose first edge lies in [a, b) begins.
"""
from __future__ import annotations

import random

import numpy as np

UNSEEN = -1


def row_lengths(frontier, offsets) -> list[int]:
    """Degree of each frontier vertex, in frontier order."""
    return [int(offsets[v + 1]) - int(offsets[v]) for v in frontier]


def running_totals(values) -> list[int]:
    """Inclusive prefix sums (entry i = values[0] + ... + values[i])."""
    return [int(x) for x in np.cumsum(np.asarray(values, dtype=np.int64))]


def chunk_size(total: int, workers: int) -> int:
    """Edges per chunk when `total` edges go to `workers` workers in nearly equal runs."""
    return -(-total // workers) if workers > 0 else 0


def chunk_starts(totals, total: int, workers: int, size: int | None = None):
    """Start of each worker's chunk as (frontier entry, edge offset in that entry's row).

    `totals` are the inclusive running totals of the frontier's degrees.  Chunk w
    covers edges [w * size, (w + 1) * size).  Rather than searching for each
    chunk's first edge, every frontier entry names the chunks that begin inside
    its own edge range (a scatter).  A chunk with no edge gets None.
    """
    size = chunk_size(total, workers) if size is None else size
    out = [None] * workers
    if size <= 0:
        return out
    lo = 0
    for entry, hi in enumerate(totals):
        hi = int(hi)
        # chunks whose first edge w * size falls in [lo, hi)
        first = -(-lo // size)
        after = -(-hi // size)
        for w in range(first, min(after, workers)):
            out[w] = (entry, w * size - lo)
        lo = hi
    return out


def scan_chunks(frontier, starts, total: int, size: int, offsets, cols, dist, claim, round_no: int,
                race=None):
    """Every worker walks its chunk of the round's edges and lists the targets it claims.

    Returns one list per worker.  With race=None the workers run one after
    another and see each other's writes.  With race=<seed> every worker sees
    the distances as they were when the round began (plus its own claims), and
    all claims are applied afterwards in a seeded random order: several workers
    may list the same vertex, and the one whose claim lands last owns it.
    """
    lists = [[] for _ in starts]
    before = list(dist) if race is not None else None
    pending = []
    for w, start in enumerate(starts):
        if start is None:
            continue
        entry, off = start
        first, stop = w * size, min((w + 1) * size, total)
        mine = set()
        pos = first
        while pos < stop:
            u = frontier[entry]
            row = int(offsets[u])
            deg = int(offsets[u + 1]) - row
            while off < deg and pos < stop:
                v = int(cols[row + off])
                if race is None:
                    fresh = dist[v] == UNSEEN
                    if fresh:
                        dist[v] = round_no
                        claim[v] = w
                else:
                    fresh = before[v] == UNSEEN and v not in mine
                    if fresh:
                        mine.add(v)
                        pending.append((w, v))
                if fresh:
                    lists[w].append(v)
                off += 1
                pos += 1
            entry += 1
            off = 0
    if race is not None:
        random.Random(race).shuffle(pending)
        for w, v in pending:
            dist[v] = round_no
            claim[v] = w
    return lists


def keep_claimed(lists, claim):
    """Worker w keeps a listed vertex only if w holds its final claim; returns the
    filtered lists and their lengths."""
    kept = [[v for v in lst if claim[v] == w] for w, lst in enumerate(lists)]
    return kept, [len(k) for k in kept]


def concatenate(lists, totals):
    """One array holding the lists in worker order; list w starts at totals[w - 1]
    (the inclusive running total of the lengths before it)."""
    out = [None] * (int(totals[-1]) if totals else 0)
    for w, lst in enumerate(lists):
        base = int(totals[w - 1]) if w > 0 else 0
        out[base:base + len(lst)] = lst
    return out


def level_synchronous_bfs(offsets, cols, source: int, workers: int, race=None, size: int | None = None):
    """Distances from `source` (-1 where unreached) by rounds of the primitives above,
    and each round's (frontier vertices, frontier edges): the work measure of the
    Analysis paragraph.  With `size` the chunk size is fixed and the worker count
    follows the round's edges; otherwise a round uses min(workers, edges) workers."""
    n = len(offsets) - 1
    dist = [UNSEEN] * n
    claim = [None] * n
    dist[source] = 0
    claim[source] = 0
    frontier = [source]
    per_round = []
    round_no = 0
    while frontier:
        round_no += 1
        totals = running_totals(row_lengths(frontier, offsets))
        edges = totals[-1]
        per_round.append((len(frontier), edges))
        active = min(workers, edges) if size is None else chunk_size(edges, size)
        if active == 0:
            break
        chunk = chunk_size(edges, active) if size is None else size
        starts = chunk_starts(totals, edges, active, chunk)
        lists = scan_chunks(frontier, starts, edges, chunk, offsets, cols, dist, claim, round_no, race)
        kept, lengths = keep_claimed(lists, claim)
        frontier = concatenate(kept, running_totals(lengths))
    return dist, per_round
