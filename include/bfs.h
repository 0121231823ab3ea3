/*
 * bfs.h -- C ABI of libbfs, a breadth-first-search library for one AMD
 * Instinct MI355X (gfx950).
 *
 * The library computes what Figure 1 of Tithi, Fogel and Chowdhury,
 * "An Optimal Level-synchronous Shared-memory Parallel BFS Algorithm"
 * (S3BFS) returns -- the distance d[0:n-1] of every vertex from a source --
 * with the paper's per-level steps (degree gather, prefix sum, splitting the
 * level's edges into equal shares, scanning, owner de-duplication and
 * linearisation of the next frontier) run as HIP kernels.  It adds a
 * deterministic parent (the smallest-id neighbour one level closer), batched
 * multi-source search and multi-root search of disjoint graphs.
 *
 * Conventions for every entry point:
 *   - The return value is a bfs_status_t: BFS_OK (0) or a negative error.
 *     No C++ exception crosses this boundary.  bfs_last_error() gives a
 *     human-readable message for the last failure on the calling thread.
 *   - "device" pointers are HIP device allocations (or host-pinned memory
 *     mapped for the device); "host" pointers are ordinary host memory.
 *   - Runs are asynchronous on the given HIP stream (a hipStream_t passed
 *     as void*; NULL is the null stream) unless stated otherwise.  A fault
 *     that happens on the device during a run is reported by bfs_sync or
 *     bfs_last_stats on that workspace before its next run (a run starts
 *     from a clean device status).
 *   - Graphs must be symmetric (undirected), with rows sorted ascending (or
 *     BFS_SORT_ROWS at bfs_init) and 0 <= cols[i] < n; n and m must fit in
 *     int32.  Self-loops and duplicate entries do not change the result.
 *     BFS_VALIDATE checks all of this.
 */
#ifndef S3BFS_BFS_H
#define S3BFS_BFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bfs_status_t;
#define BFS_OK         0
#define BFS_EINVAL    -1  /* bad argument (null pointer, bad flag, k out of range) */
#define BFS_ERANGE    -2  /* a source or root is outside [0, n) */
#define BFS_ENOMEM    -3  /* a device or host allocation failed */
#define BFS_EBADCSR   -4  /* BFS_VALIDATE found a malformed graph */
#define BFS_EHIP      -5  /* a HIP runtime call failed */
#define BFS_EOVERFLOW -6  /* batched search reached level 255 (uint8 output) */
#define BFS_EBUSY     -7  /* workspace still in flight on another stream */
#define BFS_EDEVICE   -8  /* device-side failure (a grid-barrier wait timed out) */

typedef struct bfs_graph_s* bfs_graph_t;          /* immutable device-resident CSR */
typedef struct bfs_workspace_s* bfs_workspace_t;  /* scratch for one in-flight run */

/* bfs_init flags */
#define BFS_HOST_PTRS   1u  /* offsets/cols are host memory: the library copies them */
#define BFS_DEVICE_PTRS 2u  /* offsets/cols are device memory: borrowed until bfs_graph_free */
#define BFS_VALIDATE    4u  /* check the CSR on the host (O(m log m); meant for tests) */
#define BFS_HOT_FILTER  8u  /* always build the hot-vertex filter (see bfs_init) */
#define BFS_LEAN       16u  /* never build it (no per-edge memory beyond the CSR) */
#define BFS_SORT_ROWS  32u  /* sort every row ascending first, into a copy the library owns (the
                               caller's arrays are not modified; 4 B per edge more) */

/* Execution modes (bfs_workspace_set_option(ws, BFS_OPT_MODE, ...)). */
#define BFS_MODE_AUTO        0  /* one persistent launch; small levels on a group of workgroups */
#define BFS_MODE_LEVEL       1  /* one launch pair per level, grid sized to the level's edges */
#define BFS_MODE_PLAIN       2  /* plain per-level kernel: one thread per frontier vertex */
#define BFS_MODE_INSENSITIVE 3  /* persistent, every workgroup active at every step */
#define BFS_MODE_DIRECTION   4  /* AUTO, with bottom-up levels where the frontier is large
                                   (direction optimisation; same levels and parents) */

/* Options */
#define BFS_OPT_MODE        1  /* one of BFS_MODE_* (default AUTO) */
#define BFS_OPT_SMALL_EDGES 2  /* levels with at most this many edges (capped at 16384) and at most
                                  4096 frontier vertices run on a small group of workgroups with one
                                  barrier among them per level (0 disables; default 16384) */
#define BFS_OPT_GRID        3  /* workgroups of the level loop (0 = one per 16384 edges, a multiple
                                  of 8, at least 64 and at most what the GPU holds at once) */
#define BFS_OPT_PROFILE     4  /* 1: time the main kernel with HIP events (bfs_stats_t.kernel_ms) */
#define BFS_OPT_BATCH_PULL  5  /* batched search: active edges above which a level pulls instead
                                  of pushing (-1 = never pull; default m / 8) */
#define BFS_OPT_BATCH_LEVELS 7 /* batched search: levels per replay of the captured loop (default 8) */
#define BFS_OPT_PUSH_EDGES  6  /* levels with at most this many edges push parents (atomic
                                  minimum per edge); larger ones pull them from sorted rows
                                  (default m / 24; m / 12 under BFS_MODE_LEVEL and
                                  BFS_MODE_DIRECTION) */
#define BFS_OPT_BATCH_GRAIN 8  /* batched search: edges per expansion sub-tile, the grain of
                                  the equal edge split (512, 1024 or 2048; default 1024) */
#define BFS_OPT_BATCH_TILE  9  /* batched search: vertices per tile of the dense update pass
                                  (1024, 2048 or 4096; default 2048) */
#define BFS_OPT_BU_ALPHA   10  /* BFS_MODE_DIRECTION: a level runs bottom-up when its frontier
                                  edges times alpha exceed the edges of unreached vertices
                                  (default 14) */
#define BFS_OPT_BU_BETA    11  /* BFS_MODE_DIRECTION: bottom-up stops once the frontier holds
                                  fewer than n / beta vertices (default 24) */
#define BFS_OPT_DENSE_EDGES 12 /* BFS_MODE_AUTO / INSENSITIVE: a level that pulls its parents (or
                                  has none to find) and scans at least this many edges records its
                                  new vertices as bits instead of private-queue entries and
                                  linearises them in vertex order (0 = never; default m / 24) */
#define BFS_OPT_GROUP      14  /* workgroups of that group (1..64, at most the grid; 0 = default 48) */
#define BFS_OPT_BATCH_REPLAYS 15 /* batched search: replays of the captured level loop each run
                                    enqueues before the one-workgroup finish (-1 = enough for the
                                    most levels a completed batched run of this workspace, or of any
                                    workspace on its graph, needed, 32 before the first, default;
                                    0..256 = exactly that many) */
#define BFS_OPT_HOST_STATUS 16 /* 1: every single-source or multi-root run also copies its device
                                  status into the workspace's pinned host block, on the run's
                                  stream, for bfs_run_status (default 0: no copy) */
#define BFS_OPT_SPLIT      13  /* how each level's equal shares find their start points
                                  (Analysis, Find-StartExpPoint): 0 = every frontier vertex
                                  writes itself as the start of the shares beginning inside its
                                  edge range (the paper's scatter, default); 1 = every share
                                  finds its start by a binary search of the degree prefix sums.
                                  Same result; an ablation of the cost */

typedef struct {
    int32_t levels;          /* frontiers processed: max level + 1 */
    int32_t mode;            /* BFS_MODE_* actually used */
    int32_t grid;            /* workgroups launched for the level loop */
    int32_t small_levels;    /* levels run by the group of workgroups (small levels) */
    int64_t reached;         /* vertices with a level (sum of n_l) */
    int64_t edges;           /* adjacency entries scanned (sum of e_l) */
    double  kernel_ms;       /* main-kernel time if BFS_OPT_PROFILE, else -1 */
    int32_t status;          /* device status of the run (BFS_OK or BFS_EDEVICE) */
    int32_t stats_truncated; /* 1 if more levels ran than per-level records kept */
    int32_t bottom_up_levels;/* levels run bottom-up (BFS_MODE_DIRECTION) */
} bfs_stats_t;

/*
 * Make a graph resident on the current HIP device.  An addition: the paper
 * takes the graph as given in shared memory (Figure 1 reads Degree and
 * Neighbor); on a GPU it is uploaded once and searched many times.
 *   offsets[n+1], cols[m]: CSR (int32).  With BFS_HOST_PTRS they are copied
 *   (synchronously; the call returns after the copy).  With BFS_DEVICE_PTRS
 *   the caller keeps them alive and unchanged until bfs_graph_free.
 *   stream: used for the upload.  *out receives the handle.
 *   Unless BFS_LEAN is given, graphs with m >= 2^22 (or any graph with
 *   BFS_HOT_FILTER) also get a hot-vertex filter: the 391168 vertices of
 *   highest degree (ties by id) are numbered, and an int32 per edge holds
 *   its target, or -1 minus the target's number.  Large levels then test these
 *   targets against a workgroup-local copy of their visited bits before
 *   the global visited bitmap (EXPLORE-VERTEX's visited test; results are
 *   unchanged).  This costs 4 B per edge plus 4 B
 *   per hot vertex of device memory (bfs_graph_aux_bytes) and a host pass
 *   over the degrees.
 *   With BFS_SORT_ROWS the rows need not be sorted: a device segmented sort
 *   writes a sorted copy that the graph uses (BFS_VALIDATE then checks that).
 * Errors: EINVAL (null pointers, n < 0, m < 0, both or neither pointer flag,
 *         both BFS_HOT_FILTER and BFS_LEAN), EBADCSR (BFS_VALIDATE failed),
 *         ENOMEM, EHIP.
 */
bfs_status_t bfs_init(const int32_t* offsets, const int32_t* cols, int32_t n, int64_t m,
                      uint32_t flags, void* stream, bfs_graph_t* out);

/* Release a graph (no workspace of it may be in use). */
bfs_status_t bfs_graph_free(bfs_graph_t g);

/* n and m of a resident graph. */
bfs_status_t bfs_graph_info(bfs_graph_t g, int32_t* n, int64_t* m);

/* Device bytes the library allocated for g beyond the CSR itself (the
   hot-vertex filter; 0 if it has none, and 0 for a null handle).  With
   BFS_HOST_PTRS the copied CSR is not counted. */
int64_t bfs_graph_aux_bytes(bfs_graph_t g);

/* Device bytes a workspace for up to max_sources batched sources needs
   (max_sources = 1: single-source and multi-root runs only). 0 on error.
   Its private queues are sized for BFS_MODE_AUTO with the default options
   (levels of up to m / 24 edges keep queues; larger ones are dense) and one
   root.  A run whose mode, options or roots let larger levels keep queues
   (BFS_MODE_LEVEL, BFS_MODE_DIRECTION, BFS_OPT_DENSE_EDGES = 0 or a higher
   threshold, more roots) first grows them, up to 4 B per edge. */
size_t bfs_workspace_bytes(bfs_graph_t g, int32_t max_sources);

/* Allocate a workspace (all scratch of one run).  One workspace serves one
   run at a time; give each concurrent stream its own.  Its device memory is
   one piece of bfs_workspace_bytes (plus alignment), taken from a memory pool
   the library keeps per device where the device supports stream-ordered
   allocation, on a stream of the workspace's own; creation queues the
   clearing work there and returns without waiting for the device (runs on
   any stream are ordered after it).  Errors: EINVAL, ENOMEM, EHIP. */
bfs_status_t bfs_workspace_create(bfs_graph_t g, int32_t max_sources, bfs_workspace_t* out);
/* Waits for the workspace's last run, then gives its memory back to the pool
   in stream order, without waiting for other work on the device.  The pool
   keeps up to 4 GiB of freed memory per device for later workspaces; the
   workspace's stream and pinned host block are kept for reuse too. */
bfs_status_t bfs_workspace_free(bfs_workspace_t ws);

/* Workgroups of the persistent level loop that the device holds at once: the largest useful
   BFS_OPT_GRID, and the budget that persistent runs in flight together on one device must
   share (their grids must sum to at most this, or their grid barriers can wait on each other).
   0 for a null handle. */
int32_t bfs_workspace_grid_capacity(bfs_workspace_t ws);

/* Set a BFS_OPT_* option.  EINVAL for an unknown option or bad value. */
bfs_status_t bfs_workspace_set_option(bfs_workspace_t ws, int32_t option, int64_t value);

/*
 * Single-source search (Figure 1, Parallel-BFS(s, P)).
 *   level[n] (device, int32, written): distance from source, -1 if unreached.
 *   parent[n] (device, int32, may be NULL): smallest-id neighbour one level
 *   closer; parent[source] = source; -1 if unreached.
 * The arrays are owned by the caller.  Results depend only on the graph and
 * the source, never on mode, grid, options, stream or other work in flight.
 * Asynchronous on stream in BFS_MODE_AUTO and BFS_MODE_INSENSITIVE; the
 * LEVEL and PLAIN modes read each level's size back and so synchronise.
 * Errors: EINVAL, ERANGE (source), EBUSY, EHIP; a device failure of this
 * run is reported by bfs_sync.
 */
bfs_status_t bfs_run(bfs_workspace_t ws, int32_t source, int32_t* level, int32_t* parent, void* stream);

/*
 * Multi-root search (an addition; the paper searches from one source):
 * every root starts at level 0 (host array roots[k],
 * 1 <= k <= n, repeats allowed).  With one root per component of a
 * disjoint union of graphs this runs independent searches of many small
 * graphs in one launch.  level/parent as in bfs_run (a root's parent is
 * itself; other vertices take the distance to the nearest root).
 */
bfs_status_t bfs_run_multiroot(bfs_workspace_t ws, const int32_t* roots, int32_t k,
                               int32_t* level, int32_t* parent, void* stream);

/*
 * Batched search (an addition; the paper searches from one source) of
 * k <= 256 sources (host array sources[k], repeats allowed) with
 * per-vertex 4 x 64-bit frontier/visited masks.
 *   level[n * k] (device, uint8, written): level[v * k + j] is the distance
 *   of v from sources[j], 255 if unreached.
 * The workspace must have been created with max_sources >= k.  Levels >= 255
 * do not fit: the run stops and bfs_sync returns BFS_EOVERFLOW (the int32
 * single-source path answers those sources).
 * Asynchronous on stream: the call enqueues a reset, replays of the captured
 * level loop (see BFS_OPT_BATCH_REPLAYS) and one single-workgroup kernel that
 * runs whatever levels the replays left, and returns without waiting for the
 * device; level is complete in stream order.  Device-side failures and
 * overflow are reported by bfs_sync.
 */
bfs_status_t bfs_run_batch(bfs_workspace_t ws, const int32_t* sources, int32_t k, uint8_t* level,
                           void* stream);

/*
 * Single-source search that allocates nothing, for callers that cannot
 * allocate device memory: code under HIP graph capture, serving loops that
 * must not allocate, harnesses that forbid it.  Same result as bfs_run
 * (BFS_MODE_AUTO with default options) on graph g, with no workspace: the
 * search's scratch is a fixed 64 MiB device array inside the library, one
 * per device, held from the first bfs_init on that device until the
 * process ends.
 *   level[n], parent[n] (device, int32; parent may be NULL): as in bfs_run.
 *   status (device, one int32, may be NULL): receives BFS_OK or BFS_EDEVICE
 *   when the search ends (stream-ordered), the device status bfs_sync would
 *   report for a workspace run.
 * Asynchronous on stream: the call launches kernels only (no allocation,
 * copy, memset or synchronisation), so it may be captured into a HIP graph.
 * The scratch holds what the last call left; every call on one device uses
 * the same array, so calls that overlap on a device (other streams, other
 * threads, replays of captured calls) race and must be ordered by the
 * caller.  The first call after a call on a different graph also clears the
 * scratch's frontier and queue arrays.
 * Errors: EINVAL (null graph or level), ERANGE (source), ENOMEM if the
 * graph's search needs more scratch than the array holds (about
 * 28.5 n + m / 3 bytes + 2 MiB: e.g. n = 2^20 with m up to about 100 M
 * directed entries, or n = 2^21 with m up to about 15 M, fits;
 * bfs_last_error gives both sizes), EHIP.
 */
bfs_status_t bfs_run_noalloc(bfs_graph_t g, int32_t source, int32_t* level, int32_t* parent,
                             int32_t* status, void* stream);

/* Wait for the workspace's last run; returns its device status. */
bfs_status_t bfs_sync(bfs_workspace_t ws);

/*
 * The device status of the workspace's last single-source or multi-root run
 * without waiting for anything: for callers (a server) that learn of a run's
 * completion from their own event on its stream, where a host wait on the
 * workspace would also wait for other work queued on the same hardware
 * queue.  Needs BFS_OPT_HOST_STATUS = 1 when the run was launched.  *status
 * receives BFS_OK or BFS_EDEVICE (or the run's launch error) once the run's
 * work has completed; until then the call returns BFS_EBUSY.  EINVAL for a
 * null argument, without the option, or after a batched run.  An addition:
 * the paper's search has no device of its own to fail.
 */
bfs_status_t bfs_run_status(bfs_workspace_t ws, int32_t* status);

/* Statistics of the last run (synchronises with it first). */
bfs_status_t bfs_last_stats(bfs_workspace_t ws, bfs_stats_t* out);

/* Per-level frontier sizes n_l and edge totals e_l of the last run (the
   work accounting of the paper's Analysis).  Copies min(levels, cap)
   entries into host arrays and returns the count in *count. */
bfs_status_t bfs_last_level_stats(bfs_workspace_t ws, int32_t cap, int64_t* n_l, int64_t* e_l,
                                  int32_t* count);

/* Durations (ms, HIP events on the run's stream) of the main kernel of every
   run made with BFS_OPT_PROFILE = 1 since the previous call: the persistent
   level-loop kernel (single-source and multi-root) or the level kernels of a
   batched run.  Synchronises, copies min(recorded, cap) values into ms[],
   sets *count, and forgets them.  At most 4096 runs are remembered. */
bfs_status_t bfs_kernel_times(bfs_workspace_t ws, int32_t cap, double* ms, int32_t* count);

/* Per-level device time of the last run in BFS_MODE_AUTO or INSENSITIVE:
   expand_us[l] from the start of level l to the end of its scan of the
   adjacency (the whole level when it ran on one workgroup up to its own
   de-duplication), compact_us[l] for its de-duplication and linearisation.
   Read from the device's 100 MHz clock by workgroup 0; count = 0 for the
   host-paced modes.  Synchronises with the run. */
bfs_status_t bfs_last_level_times(bfs_workspace_t ws, int32_t cap, double* expand_us, double* compact_us,
                                  int32_t* count);

const char* bfs_status_str(bfs_status_t s);
const char* bfs_last_error(void);

/* ---- autotuning ------------------------------------------------------------------------ */

/*
 * Launch shape chosen for one workspace and its graph.  The grain of the
 * equal edge split (Figure 1, Find-StartExpPoint: shares of a fixed number
 * of edges) and the tile shapes are free parameters of the method; the
 * tuner picks them by timing real runs.
 */
typedef struct {
    int32_t batch_grain;   /* BFS_OPT_BATCH_GRAIN */
    int32_t batch_tile;    /* BFS_OPT_BATCH_TILE */
    int32_t batch_levels;  /* BFS_OPT_BATCH_LEVELS */
    int32_t batch_pull;    /* BFS_OPT_BATCH_PULL (-1 = never pull) */
    int32_t grid;          /* BFS_OPT_GRID (0 = sized to the graph) */
    int32_t small_edges;   /* BFS_OPT_SMALL_EDGES */
    int32_t push_edges;    /* BFS_OPT_PUSH_EDGES */
    int32_t dense_edges;   /* BFS_OPT_DENSE_EDGES */
    int32_t trials;        /* configurations timed by the last bfs_autotune */
    double  default_ms;    /* one pass over the sample with the settings the call started from */
    double  best_ms;       /* one pass over the sample with the chosen settings */
} bfs_tune_t;

#define BFS_TUNE_BATCH  1u  /* tune the batched launch: grain, update tile, pull threshold, replay length */
#define BFS_TUNE_SINGLE 2u  /* tune single-source runs: grid, group-level, push and dense thresholds */

/*
 * Times candidate settings on the workspace's own graph and keeps the
 * fastest (coordinate descent: grain and tile together, then each
 * threshold in turn; each candidate is run once untimed, then three times,
 * and its median wall time counts).  sources: host array of k vertices.
 * BFS_TUNE_BATCH runs them as one batch (2 <= k <= max_sources);
 * BFS_TUNE_SINGLE runs each with levels and parents (1 <= k <= 64).  The
 * chosen settings are applied to ws and written to *out (which may be
 * NULL); results do not depend on them.  Allocates and frees temporary
 * output arrays; synchronous; do not call while ws is in flight elsewhere.
 * Errors: EINVAL (bad arguments), ERANGE (a source outside [0, n)), or a
 * run's error.
 */
bfs_status_t bfs_autotune(bfs_workspace_t ws, const int32_t* sources, int32_t k, uint32_t what, bfs_tune_t* out);

/* The workspace's current settings, in the same form (trials and times 0). */
bfs_status_t bfs_workspace_get_tuning(bfs_workspace_t ws, bfs_tune_t* out);

#ifdef __cplusplus
}
#endif

#endif /* S3BFS_BFS_H */
