/*
 * bfs_test.h -- entry points of libbfs that serve its tests and its
 * measurements, not its users: one primitive of the level loop run on its
 * own, a kernel that measures the device's random-probe rate, and a time
 * limit for the level loop's waits that tests of failure handling shorten.
 * They follow the conventions of bfs.h (status codes, device pointers,
 * streams).
 */
#ifndef S3BFS_BFS_TEST_H
#define S3BFS_BFS_TEST_H

#include "bfs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- primitives of the level loop, exposed for testing ------------------------------ */

/*
 * Owner de-duplication and linearisation of one level (Figure 1: keep a
 * private-queue entry v of queue i only if Owner[v] = i, prefix-sum the
 * queue sizes, copy the survivors to the next CurLevelVertices), fused with
 * the next level's degree gather, degree prefix sum and share start points
 * (Find-StartExpPoint).  All pointers are device memory.
 *   cand[ntiles * grain], cnt[ntiles]: tile t's private queue is
 *     cand[t*grain .. t*grain + cnt[t]); its entries' slot ids are their
 *     positions in cand.
 *   owner[n]: slot id that owns each vertex.
 *   offsets[n+1]: graph CSR offsets (degree = offsets[v+1] - offsets[v]).
 *   Outputs: out_v[i] = v_i, the i-th survivor; out_rs[i] = offsets[v_i];
 *   out_ex[i] = sum of the degrees of the
 *   survivors before i (in output order), out_ex[count] = total;
 *   out_tstart[t] = index of the survivor holding edge t*grain (tstart_cap
 *   entries available; BFS_EDEVICE if the edge total needs more);
 *   totals[0] = survivor count (degree >= 1 only), totals[1] = edge total
 *   (int32 device array of 2).  Survivors of degree 0 are dropped.
 *   out_v and out_rs need n entries, out_ex n + 1.  Output order is unspecified;
 *   the set is exact.  Synchronises with stream.
 * grain must be the library's tile size (bfs_prim_grain()).
 */
bfs_status_t bfs_prim_compact(const int32_t* offsets, int32_t n, const int32_t* owner,
                              const int32_t* cand, const int32_t* cnt, int32_t ntiles,
                              int32_t* out_v, int32_t* out_rs, int32_t* out_ex, int32_t* out_tstart,
                              int32_t tstart_cap, int32_t* totals, void* stream);

/* Edges per share (tile) of the multi-workgroup level loop. */
int32_t bfs_prim_grain(void);

/* ---- measurement aid ---------------------------------------------------------------- */

/*
 * Random-probe ceiling.  The expansion step (Figure 1, EXPLORE-VERTEX)
 * streams the column array and probes per-vertex state at the neighbour
 * ids it reads.  This kernel reproduces that access pattern alone: it
 * streams idx[0 .. count) and, for each entry v, reads table[v >> shift]
 * (shift 5: a bit of a bitmap of 32-bit words, as the visited filter;
 * shift 0: a 32-bit entry, as the level array); entries outside
 * [0, table_words) are skipped.  All pointers are device memory; *sink
 * receives nothing unless a checksum hits a fixed value (it only keeps the
 * reads alive).  Asynchronous on stream: time it with events there.
 * EINVAL for a null pointer, count < 0, table_words < 1 or shift outside
 * [0, 5]; EHIP if the launch fails.
 */
bfs_status_t bfs_probe_rate_kernel(const int32_t* idx, int64_t count, const uint32_t* table,
                                   int64_t table_words, int32_t shift, int32_t* sink, void* stream);

/* ---- failure handling ----------------------------------------------------------------- */

/*
 * Time limit, in ticks of the 100 MHz device clock, of every wait in the
 * persistent level loop of ws's single-source and multi-root runs
 * (BFS_MODE_AUTO, BFS_MODE_INSENSITIVE, BFS_MODE_DIRECTION: grid, XCD and
 * group barriers, look-back over the shares; per-level launches and batched
 * runs keep the default).  A wait that sees no progress for that long
 * records a device failure, every workgroup then leaves the kernel at its
 * next wait, and the run reports BFS_EDEVICE (bfs_sync, bfs_last_stats);
 * the next run starts clean.  ticks = 0 restores the default (3 s).  For
 * tests that force that path without faulting or hanging the device.
 * EINVAL for a null workspace.
 */
bfs_status_t bfs_workspace_set_spin_ticks(bfs_workspace_t ws, uint64_t ticks);

#ifdef __cplusplus
}
#endif

#endif /* S3BFS_BFS_TEST_H */
