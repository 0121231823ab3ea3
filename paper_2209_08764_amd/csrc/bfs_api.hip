// C ABI of libbfs: graph residency, workspaces and run orchestration.
// The entry points are declared and documented in include/bfs.h (users) and
// include/bfs_test.h (test and measurement aids).
#include "../../include/bfs_test.h"
#include "bfs_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace s3bfs;

namespace {

thread_local std::string g_last_error;

bfs_status_t fail(bfs_status_t code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(BFS_EHIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

constexpr uint64_t kSpinTicks = 300000000ull;  // 3 s at the 100 MHz s_memrealtime clock
// Default split of levels by their edges: up to m / kLevelSplit a level pushes
// its parents (an atomic minimum per edge into an unsettled vertex); above it
// the level pulls them from sorted rows and keeps its new vertices as bits.
// Pushing pays for small levels; a level of a few thousand hubs with tens of
// millions of edges is cheaper pulled, since each new vertex finds a hub a few
// entries into its row.  Measured on R-MAT scale 24 over 64 sources (harmonic
// mean GTEPS): m / 12 65.4, m / 24 66.4, m / 32 66.3, m / 48 66.1, m / 96 65.1.
// Per-level launches and direction optimisation have no dense levels, and
// their pulls test the level array, so they keep pushing up to m / 12.
constexpr int64_t kLevelSplit = 24;
constexpr int64_t kLevelSplitNoDense = 12;

template <typename T>
hipError_t dalloc(T** p, size_t count) {
    return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
}

// Entries of the private-queue array that a run needs.  Share b of a level
// keeps its queue in cand[tb * kGrain, te * kGrain), so a level that keeps
// queues needs its edges rounded up to whole sub-tiles.  Dense levels keep
// none, so with the default thresholds only levels up to m / kLevelSplit edges do;
// per-level launches, direction optimisation (whose bottom-up levels queue up
// to n vertices) and dense levels switched off may queue any level.  The
// roots sit there as the queues of level -1.
int64_t cand_need(int64_t m, int64_t n, int32_t mode, int64_t push_edges, int64_t dense_edges, int64_t small_edges,
                  int64_t nroots, bool parents) {
    if (mode == BFS_MODE_PLAIN) return kGrain;  // the plain comparator keeps no queues
    int64_t e;
    if (mode == BFS_MODE_LEVEL || mode == BFS_MODE_DIRECTION || dense_edges <= 0) e = std::max(m, n);
    else e = std::min(std::max(parents ? push_edges : 0, dense_edges - 1), m);
    (void)small_edges;  // group levels append to their own arrays
    auto tiles = [](int64_t x) { return (x + kGrain - 1) / kGrain; };
    return std::max<int64_t>({tiles(e), tiles(nroots), 1}) * kGrain;
}

// Private-queue entries a workspace starts with: enough for BFS_MODE_AUTO with
// the default options, parents and one root.
int64_t default_cand(int64_t m, int64_t n) {
    const int64_t split = std::min<int64_t>(m / kLevelSplit, INT32_MAX);
    return cand_need(m, n, BFS_MODE_AUTO, split, std::max<int64_t>(split, 1), kDefaultSmallEdges, 1, true);
}

}  // namespace

struct bfs_graph_s {
    int device = 0;
    int32_t n = 0;
    int64_t m = 0;
    int32_t* offsets = nullptr;
    int32_t* cols = nullptr;
    bool owned = false;         // offsets and cols are the library's copies
    bool owned_cols = false;    // cols is the library's (rows sorted from the caller's)
    int32_t* colx = nullptr;    // hot-vertex filter: each edge's target, or -1 - its hot number
    int32_t* hot_vid = nullptr; // vertex id of each hot number
    int32_t hot_count = 0;      // hot vertices
    int32_t hot_words = 0;      // words of a workspace's hot-bit arrays (0: no filter)
    uint64_t uid = 0;           // distinct for every graph made resident in this process
    std::atomic<int32_t> batch_depth{0};  // most levels a completed batched run on it needed
};

struct bfs_workspace_s {
    bfs_graph_s* g = nullptr;
    int device = 0;
    int32_t max_sources = 1;
    int32_t max_tiles = 0;
    // device memory: one arena, from the library's stream-ordered pool where the device has one
    void* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    bool arena_pooled = false;
    int32_t* cand_grown = nullptr;  // a private-queue array that outgrew the arena's
    bool cand_pooled = false;
    int64_t cand_cap = 0;   // entries of the private-queue array (grown when a run needs more)
    int32_t grid_cap = 0;
    // single-source buffers
    uint32_t* bitmap = nullptr;
    uint32_t* hot[2] = {nullptr, nullptr};
    uint32_t* fbits[2] = {nullptr, nullptr};
    uint32_t* snap = nullptr;
    int32_t* owner = nullptr;
    int32_t* f_rs[2] = {nullptr, nullptr};
    int32_t* f_ex[2] = {nullptr, nullptr};
    int32_t* f_v[2] = {nullptr, nullptr};
    int32_t* tstart[2] = {nullptr, nullptr};
    int32_t* cand = nullptr;
    int32_t* cnt = nullptr;
    unsigned long long* desc[2] = {nullptr, nullptr};
    Ctrl* ctrl = nullptr;
    XBar* xbar = nullptr;
    Aux* aux = nullptr;
    int32_t* stat_nl = nullptr;
    int32_t* stat_el = nullptr;
    uint64_t* stat_ts = nullptr;
    int32_t* roots = nullptr;
    int32_t* plain_fv[2] = {nullptr, nullptr};
    int32_t* gv[2] = {nullptr, nullptr};   // group levels' frontier entries
    int32_t* grs[2] = {nullptr, nullptr};
    int32_t* gd[2] = {nullptr, nullptr};
    // batched buffers
    unsigned long long* b_fr = nullptr;
    unsigned long long* b_nx = nullptr;
    unsigned long long* b_vis = nullptr;
    int32_t* b_act[2] = {nullptr, nullptr};
    int32_t* b_act_rs[2] = {nullptr, nullptr};
    int32_t* b_act_ex[2] = {nullptr, nullptr};
    int32_t* b_tstart[2] = {nullptr, nullptr};
    unsigned long long* b_desc[2] = {nullptr, nullptr};
    uint32_t* b_act_bits = nullptr;
    unsigned long long* b_fr_hot = nullptr;  // hot vertices' frontier masks (graphs with hot numbering)
    int32_t* b_nz_v = nullptr;
    int32_t* b_nz_ts = nullptr;
    int32_t* b_sources = nullptr;
    int32_t b_max_tiles = 0;
    int32_t b_utiles = 0;
    int32_t b_desc_cap = 0;
    int32_t b_grid_cap = 0;
    int32_t b_bvt = kBVTDefault;         // edges per thread of an expansion sub-tile
    int32_t b_uv = kUVDefault;           // vertices per thread of an update tile
    int32_t batch_levels = 8;            // levels per replay of the captured loop
    int32_t batch_replays = -1;          // replays per run (-1: enough for the deepest run seen)
    int32_t b_seen = 0;                  // most levels a completed batched run needed (0: none yet)
    bool last_batch = false;             // the last run was batched
    hipStream_t own_stream = nullptr;    // the workspace's private stream (set-up and capture)
    hipGraphExec_t b_exec = nullptr;
    hipGraph_t b_graph = nullptr;
    BatchArgs* b_args = nullptr;         // per-run arguments the captured kernels read
    // host side
    Ctrl* h_ctrl = nullptr;  // pinned
    hipEvent_t ev_done = nullptr, ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_ready = nullptr;  // the set-up work queued on own_stream at creation
    bool init_pending = false;      // runs on other streams still have to wait for it
    hipStream_t last_stream = nullptr;
    bool has_run = false;
    bool profiled = false;
    int32_t mode = BFS_MODE_AUTO;
    int32_t small_edges = kDefaultSmallEdges;
    int32_t group = kGroupMax;
    int32_t bu_alpha = 14;
    int32_t bu_beta = 24;
    int32_t push_edges = -1;  // -1: m / kLevelSplit of the workspace's graph
    int32_t dense_edges = -1; // -1: m / kLevelSplit of the workspace's graph
    int32_t grid_opt = 0;
    int32_t profile = 0;
    int32_t batch_pull = -2;  // -2: library default
    int32_t split_search = 0; // BFS_OPT_SPLIT
    uint64_t spin_ticks = 0;  // time limit of the persistent loop's waits (0: kSpinTicks); tests only
    bool host_status_copy = false;  // BFS_OPT_HOST_STATUS
    bool status_copied = false;  // the last run copied its status to h_ctrl->error
    // last run
    int32_t last_mode = 0;
    int32_t last_grid = 0;
    bool host_stats = false;
    std::vector<int64_t> h_nl, h_el;
    int32_t host_status = BFS_OK;
    // BFS_OPT_PROFILE: event pairs around the main kernel of each run
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
    size_t prof_used = 0;
};

namespace {

// ---- workspace memory ---------------------------------------------------------------------
// A workspace's device arrays are slices of one arena.  Where the device supports
// stream-ordered allocation the arena comes from a pool the library keeps per device and is
// allocated and freed on the workspace's own stream, so creating or dropping a workspace waits
// for nothing else in flight (a plain hipFree may wait for the whole device); freed arenas stay
// in the pool, up to kPoolKeep bytes per device, for the next workspace.
constexpr int kPoolDevices = 64;
constexpr uint64_t kPoolKeep = uint64_t(4) << 30;
constexpr size_t kSliceAlign = 256;

struct ArenaPools {
    std::mutex mu;
    hipMemPool_t pool[kPoolDevices] = {};
    bool tried[kPoolDevices] = {};
};
ArenaPools g_pools;

hipMemPool_t arena_pool(int device) {
    if (device < 0 || device >= kPoolDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_pools.mu);
    if (!g_pools.tried[device]) {
        g_pools.tried[device] = true;
        int supported = 0;
        if (hipDeviceGetAttribute(&supported, hipDeviceAttributeMemoryPoolsSupported, device) == hipSuccess &&
            supported) {
            hipMemPoolProps props;
            std::memset(&props, 0, sizeof(props));
            props.allocType = hipMemAllocationTypePinned;
            props.handleTypes = hipMemHandleTypeNone;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = device;
            hipMemPool_t pool = nullptr;
            if (hipMemPoolCreate(&pool, &props) == hipSuccess) {
                uint64_t keep = kPoolKeep;
                (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
                g_pools.pool[device] = pool;
            }
        }
    }
    return g_pools.pool[device];
}

// Device memory of `bytes` on `stream`'s device: from the pool (*pooled = true), ready in stream
// order on `stream` (work on other streams must be ordered after it: workspaces do so through
// ev_ready), or, without a pool, from hipMalloc.
hipError_t pool_alloc(int device, hipStream_t stream, size_t bytes, void** out, bool* pooled) {
    *out = nullptr;
    *pooled = false;
    if (hipMemPool_t pool = arena_pool(device)) {
        if (hipMallocFromPoolAsync(out, bytes, pool, stream) == hipSuccess) {
            *pooled = true;
            return hipSuccess;
        }
        *out = nullptr;
    }
    return hipMalloc(out, bytes);
}

void pool_free(void* ptr, bool pooled, hipStream_t stream) {
    if (!ptr) return;
    if (pooled) (void)hipFreeAsync(ptr, stream);
    else (void)hipFree(ptr);
}

// The next aligned slice of the workspace's arena for `count` elements.
template <typename T>
hipError_t take(bfs_workspace_s* ws, T** p, size_t count) {
    const size_t b = (std::max<size_t>(count, 1) * sizeof(T) + kSliceAlign - 1) / kSliceAlign * kSliceAlign;
    *p = nullptr;
    if (!ws->arena || ws->arena_used + b > ws->arena_bytes) return hipErrorOutOfMemory;
    *p = reinterpret_cast<T*>(static_cast<unsigned char*>(ws->arena) + ws->arena_used);
    ws->arena_used += b;
    return hipSuccess;
}

// Pinned host copies of the control block: hipHostFree can wait for the whole device, so a
// dropped workspace's block goes to a free list for the next workspace instead.
struct PinnedCtrl {
    std::mutex mu;
    std::vector<Ctrl*> free;
};
PinnedCtrl g_pinned;

hipError_t pinned_ctrl_take(Ctrl** p) {
    {
        std::lock_guard<std::mutex> lk(g_pinned.mu);
        if (!g_pinned.free.empty()) {
            *p = g_pinned.free.back();
            g_pinned.free.pop_back();
            return hipSuccess;
        }
    }
    return hipHostMalloc(reinterpret_cast<void**>(p), sizeof(Ctrl), hipHostMallocPortable);  // any device may reuse it
}

void pinned_ctrl_give(Ctrl* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pinned.mu);
    g_pinned.free.push_back(p);
}

// Workspace streams are kept too: destroying one waits for the work queued on it (the arena's
// stream-ordered free among it), which can sit behind other streams' kernels on a shared
// hardware queue.  A dropped workspace's stream serves the next workspace on its device.
struct StreamPool {
    std::mutex mu;
    std::vector<hipStream_t> free[kPoolDevices];
};
StreamPool g_streams;

hipError_t stream_take(int device, hipStream_t* s) {
    if (device >= 0 && device < kPoolDevices) {
        std::lock_guard<std::mutex> lk(g_streams.mu);
        auto& f = g_streams.free[device];
        if (!f.empty()) {
            *s = f.back();
            f.pop_back();
            return hipSuccess;
        }
    }
    return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}

void stream_give(int device, hipStream_t s) {
    if (!s) return;
    if (device < 0 || device >= kPoolDevices) {
        (void)hipStreamDestroy(s);
        return;
    }
    std::lock_guard<std::mutex> lk(g_streams.mu);
    g_streams.free[device].push_back(s);
}

// Orders a run on stream s after the workspace's set-up (queued on its own stream at creation).
bfs_status_t wait_ready(bfs_workspace_s* ws, hipStream_t s) {
    if (!ws->init_pending) return BFS_OK;
    HIP_TRY(hipStreamWaitEvent(s, ws->ev_ready, 0));
    if (hipEventQuery(ws->ev_ready) == hipSuccess) ws->init_pending = false;
    return BFS_OK;
}

bfs_status_t validate_csr(const int32_t* off, const int32_t* cols, int32_t n, int64_t m) {
    if (off[0] != 0) return fail(BFS_EBADCSR, "offsets[0] = %d, expected 0", off[0]);
    if ((int64_t)off[n] != m) return fail(BFS_EBADCSR, "offsets[n] = %d but m = %lld", off[n], (long long)m);
    for (int32_t v = 0; v < n; ++v)
        if (off[v + 1] < off[v]) return fail(BFS_EBADCSR, "offsets decrease at vertex %d", v);
    for (int64_t e = 0; e < m; ++e)
        if (cols[e] < 0 || cols[e] >= n) return fail(BFS_EBADCSR, "cols[%lld] = %d out of range", (long long)e, cols[e]);
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = off[v] + 1; e < off[v + 1]; ++e)
            if (cols[e] < cols[e - 1]) return fail(BFS_EBADCSR, "row %d is not sorted", v);
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            const int32_t v = cols[e];
            if (!std::binary_search(cols + off[v], cols + off[v + 1], u))
                return fail(BFS_EBADCSR, "edge (%d,%d) has no reverse: graph is not symmetric", u, v);
        }
    return BFS_OK;
}

int32_t dense_edges_of(const bfs_workspace_s* ws) {
    return ws->dense_edges >= 0 ? ws->dense_edges
                                : (int32_t)std::min<int64_t>(std::max<int64_t>(ws->g->m / kLevelSplit, 1), INT32_MAX);
}

int32_t push_edges_of(const bfs_workspace_s* ws) {
    const bool no_dense = ws->mode == BFS_MODE_DIRECTION || ws->mode == BFS_MODE_LEVEL;
    const int64_t split = no_dense ? kLevelSplitNoDense : kLevelSplit;
    return ws->push_edges >= 0 ? ws->push_edges : (int32_t)std::min<int64_t>(ws->g->m / split, INT32_MAX);
}

// Private-queue entries a run of ws with its current mode and options needs.
int64_t ws_cand_need(const bfs_workspace_s* ws, int64_t nroots, bool parents) {
    return cand_need(ws->g->m, ws->g->n, ws->mode, push_edges_of(ws), dense_edges_of(ws), ws->small_edges, nroots,
                     parents);
}

// Grows the private-queue array when this run's mode, options or roots need more
// than it holds (after the workspace's last run has finished with it).
bfs_status_t ensure_cand(bfs_workspace_s* ws, int64_t need) {
    if (need <= ws->cand_cap) return BFS_OK;
    if (ws->has_run) HIP_TRY(hipEventSynchronize(ws->ev_done));
    void* grown = nullptr;
    bool pooled = false;
    if (pool_alloc(ws->device, ws->own_stream, sizeof(int32_t) * (size_t)need, &grown, &pooled) != hipSuccess)
        return fail(BFS_ENOMEM, "growing the private queues to %lld entries failed", (long long)need);
    hipError_t e = hipMemsetAsync(grown, 0, sizeof(int32_t) * (size_t)need, ws->own_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ws->own_stream);
    if (e != hipSuccess) {
        pool_free(grown, pooled, ws->own_stream);
        return fail(BFS_EHIP, "clearing the private queues: %s", hipGetErrorString(e));
    }
    pool_free(ws->cand_grown, ws->cand_pooled, ws->own_stream);  // the arena's slice just goes unused
    ws->cand_grown = ws->cand = static_cast<int32_t*>(grown);
    ws->cand_pooled = pooled;
    ws->cand_cap = need;
    return BFS_OK;
}

Params make_params(bfs_workspace_s* ws, int32_t* level, int32_t* parent) {
    Params p{};
    p.offsets = ws->g->offsets;
    p.cols = ws->g->cols;
    p.colx = ws->g->colx;
    p.hot_vid = ws->g->hot_vid;
    p.hot_count = ws->g->colx ? ws->g->hot_count : 0;
    p.hot[0] = ws->hot[0];
    p.hot[1] = ws->hot[1];
    p.hot_words = ws->g->colx ? ws->g->hot_words : 0;
    p.fbits[0] = ws->fbits[0];
    p.fbits[1] = ws->fbits[1];
    p.snap = ws->snap;
    p.direction = ws->mode == BFS_MODE_DIRECTION;
    p.bu_alpha = ws->bu_alpha;
    p.bu_beta = ws->bu_beta;
    p.n = ws->g->n;
    p.m = ws->g->m;
    p.level = level;
    p.parent = parent;
    p.bitmap = ws->bitmap;
    p.owner = ws->owner;
    for (int i = 0; i < 2; ++i) {
        p.f_rs[i] = ws->f_rs[i];
        p.f_ex[i] = ws->f_ex[i];
        p.f_v[i] = ws->f_v[i];
        p.tstart[i] = ws->tstart[i];
        p.desc[i] = ws->desc[i];
    }
    p.cand = ws->cand;
    p.cand_cap = ws->cand_cap;
    p.cnt = ws->cnt;
    p.ctrl = ws->ctrl;
    p.xbar = ws->xbar;
    p.aux = ws->aux;
    p.stat_nl = ws->stat_nl;
    p.stat_el = ws->stat_el;
    p.stat_ts = ws->stat_ts;
    p.small_edges = ws->small_edges;
    p.group = ws->group;
    for (int i = 0; i < 2; ++i) {
        p.gv[i] = ws->gv[i];
        p.grs[i] = ws->grs[i];
        p.gd[i] = ws->gd[i];
    }
    // Pushing costs one atomic per scanned edge into an unsettled vertex; pulling
    // costs about one row read per new vertex but long ones when the frontier is
    // small next to what it discovers.  Levels below an eighth of the graph push.
    p.push_edges = push_edges_of(ws);
    p.max_tiles = ws->max_tiles;
    p.split_search = ws->split_search;
    p.spin_ticks = kSpinTicks;
    return p;
}

bfs_status_t check_busy(bfs_workspace_s* ws, hipStream_t s) {
    if (ws->has_run && ws->last_stream != s) {
        hipError_t q = hipEventQuery(ws->ev_done);
        if (q == hipErrorNotReady) return fail(BFS_EBUSY, "workspace still running on another stream");
        if (q != hipSuccess) return fail(BFS_EHIP, "hipEventQuery: %s", hipGetErrorString(q));
    }
    return BFS_OK;
}

// Workgroups of the level loop.  By default the grid follows the graph: one
// workgroup per kEdgesPerWg edges (a multiple of 8, so that every XCD gets as
// many), at least kMinGrid and at most what fits on the GPU at once.  A level
// cannot use more workgroups than it has 2048-edge sub-tiles, and every extra
// workgroup lengthens each grid barrier.
int default_grid(int cap, int64_t m) {
    constexpr int64_t kEdgesPerWg = 16384, kMinGrid = 64;
    const int64_t want = std::max<int64_t>(kMinGrid, (m / kEdgesPerWg + 7) / 8 * 8);
    return std::max(1, (int)std::min<int64_t>(cap, want));
}

int grid_for(bfs_workspace_s* ws) {
    if (ws->grid_opt > 0) return std::max(1, std::min(ws->grid_cap, ws->grid_opt));
    return default_grid(ws->grid_cap, ws->g->m);
}

bfs_status_t read_ctrl(bfs_workspace_s* ws, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(ws->h_ctrl, ws->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return BFS_OK;
}

// Level loop driven from the host: one expand and one compact launch per
// level, each with a grid sized to the level's shares.
bfs_status_t run_level_mode(bfs_workspace_s* ws, Params& p, hipStream_t s) {
    const int rtiles = (p.nroots + kGrain - 1) / kGrain;
    const int gmax = grid_for(ws);
    const int pr = std::min(rtiles, gmax);
    HIP_TRY(launch_prep(p, pr, p.parent != nullptr, s));
    HIP_TRY(launch_level_roots(p, pr, s));
    HIP_TRY(launch_level_compact(p, -1, rtiles, pr, s));
    ws->h_nl.clear();
    ws->h_el.clear();
    for (int l = 0;; ++l) {
        bfs_status_t st = read_ctrl(ws, s);
        if (st) return st;
        if (ws->h_ctrl->error) return fail(BFS_EDEVICE, "device-side failure (code %d)", ws->h_ctrl->error);
        const int par = l & 1;
        const int n_l = ws->h_ctrl->nl[par], e_l = ws->h_ctrl->el[par], kept = ws->h_ctrl->kept[par];
        if (kept > 0) {
            ws->h_nl.push_back(kept);
            ws->h_el.push_back(e_l);
        }
        if (n_l == 0) break;
        const int ntiles = (int)(((int64_t)e_l + kGrain - 1) / kGrain);
        const int shares = std::min(ntiles, gmax);  // P_l = min(P, W_l)
        HIP_TRY(launch_level_expand(p, l, ntiles, shares, s));
        HIP_TRY(launch_level_compact(p, l, ntiles, shares, s));
    }
    ws->host_stats = true;
    ws->last_grid = gmax;
    return BFS_OK;
}

// Plain per-level kernel: one thread per frontier vertex, no edge split.
bfs_status_t run_plain_mode(bfs_workspace_s* ws, Params& p, hipStream_t s) {
    const int32_t n = ws->g->n;
    if (!ws->plain_fv[0]) {
        HIP_TRY(dalloc(&ws->plain_fv[0], (size_t)n + 1));
        HIP_TRY(dalloc(&ws->plain_fv[1], (size_t)n + 1));
    }
    if (p.roots) return fail(BFS_EINVAL, "BFS_MODE_PLAIN runs single-source searches only");
    HIP_TRY(launch_prep(p, 0, false, s));
    HIP_TRY(launch_plain_init(p, ws->plain_fv[0], s));
    ws->h_nl.clear();
    ws->h_el.clear();
    int nf = 1;
    for (int l = 0; nf > 0; ++l) {
        ws->h_nl.push_back(nf);
        ws->h_el.push_back(-1);
        HIP_TRY(hipMemsetAsync(&ws->ctrl->plain_next, 0, sizeof(int), s));
        HIP_TRY(launch_plain_level(p, l, ws->plain_fv[l & 1], nf, ws->plain_fv[(l + 1) & 1], s));
        bfs_status_t st = read_ctrl(ws, s);
        if (st) return st;
        nf = ws->h_ctrl->plain_next;
    }
    if (p.parent) HIP_TRY(launch_parent(p, s));
    ws->host_stats = true;
    ws->last_grid = 0;
    return BFS_OK;
}

constexpr size_t kProfCap = 4096;

// Next free event pair for a profiled run (created on first use).
bfs_status_t profile_slot(bfs_workspace_s* ws, std::pair<hipEvent_t, hipEvent_t>** out) {
    if (ws->prof_used >= kProfCap) return fail(BFS_EINVAL, "more than %zu profiled runs without bfs_kernel_times", kProfCap);
    if (ws->prof_used == ws->prof_ev.size()) {
        hipEvent_t a, b;
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        ws->prof_ev.emplace_back(a, b);
    }
    *out = &ws->prof_ev[ws->prof_used++];
    return BFS_OK;
}

bfs_status_t run_common(bfs_workspace_s* ws, const int32_t* roots_host, int32_t k, int32_t single,
                        int32_t* level, int32_t* parent, void* stream) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!ws) return fail(BFS_EINVAL, "null workspace");
    if (!level) return fail(BFS_EINVAL, "null level array");
    bfs_status_t st = check_busy(ws, s);
    if (st) return st;
    HIP_TRY(hipSetDevice(ws->device));
    if (roots_host && (k < 1 || k > ws->g->n)) return fail(BFS_EINVAL, "need 1 <= k <= n roots");
    if ((st = wait_ready(ws, s))) return st;
    st = ensure_cand(ws, ws_cand_need(ws, roots_host ? k : 1, parent != nullptr));
    if (st) return st;
    Params p = make_params(ws, level, parent);
    if (roots_host) {
        for (int32_t i = 0; i < k; ++i)
            if (roots_host[i] < 0 || roots_host[i] >= ws->g->n)
                return fail(BFS_ERANGE, "root %d = %d outside [0, %d)", i, roots_host[i], ws->g->n);
        HIP_TRY(hipMemcpyAsync(ws->roots, roots_host, sizeof(int32_t) * (size_t)k, hipMemcpyHostToDevice, s));
        p.roots = ws->roots;
        p.nroots = k;
    } else {
        if (single < 0 || single >= ws->g->n) return fail(BFS_ERANGE, "source %d outside [0, %d)", single, ws->g->n);
        p.roots = nullptr;
        p.single_root = single;
        p.nroots = 1;
    }
    ws->host_stats = false;
    ws->profiled = false;
    ws->last_mode = ws->mode;
    ws->host_status = BFS_OK;
    ws->last_batch = false;
    int mode = ws->mode;
    if (mode == BFS_MODE_LEVEL) {
        st = run_level_mode(ws, p, s);
    } else if (mode == BFS_MODE_PLAIN) {
        st = run_plain_mode(ws, p, s);
    } else {
        if (mode == BFS_MODE_INSENSITIVE) {
            p.small_edges = 0;
            p.insensitive = 1;
        }
        p.fb_pull = !p.direction && p.parent != nullptr;
        p.dense_edges = p.direction ? 0 : dense_edges_of(ws);
        if (ws->spin_ticks) p.spin_ticks = ws->spin_ticks;
        const int grid = grid_for(ws);
        const int rtiles = (p.nroots + kGrain - 1) / kGrain;
        HIP_TRY(launch_prep(p, std::min(rtiles, grid), p.parent != nullptr, s));
        std::pair<hipEvent_t, hipEvent_t>* pe = nullptr;
        if (ws->profile) {
            st = profile_slot(ws, &pe);
            if (st) return st;
            HIP_TRY(hipEventRecord(pe->first, s));
        }
        HIP_TRY(launch_persistent(p, grid, s));
        if (pe) {
            HIP_TRY(hipEventRecord(pe->second, s));
            ws->profiled = true;
        }
        ws->last_grid = grid;
        st = BFS_OK;
    }
    ws->host_status = st;
    // the run's device status into the pinned block, in stream order, for bfs_run_status
    ws->status_copied = false;
    if (st == BFS_OK && ws->host_status_copy) {
        HIP_TRY(hipMemcpyAsync(&ws->h_ctrl->error, &ws->ctrl->error, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        ws->status_copied = true;
    }
    HIP_TRY(hipEventRecord(ws->ev_done, s));
    ws->last_stream = s;
    ws->has_run = true;
    return st;
}

BatchParams make_batch_params(bfs_workspace_s* ws) {
    BatchParams bp{};
    bp.offsets = ws->g->offsets;
    bp.cols = ws->g->cols;
    bp.n = ws->g->n;
    bp.m = ws->g->m;
    bp.args = ws->b_args;
    bp.fr = ws->b_fr;
    bp.nx = ws->b_nx;
    bp.vis = ws->b_vis;
    for (int i = 0; i < 2; ++i) {
        bp.act[i] = ws->b_act[i];
        bp.act_rs[i] = ws->b_act_rs[i];
        bp.act_ex[i] = ws->b_act_ex[i];
        bp.act_ts[i] = ws->b_tstart[i];
        bp.desc[i] = ws->b_desc[i];
    }
    bp.act_bits = ws->b_act_bits;
    bp.colx = ws->g->colx;
    bp.hot_vid = ws->g->hot_vid;
    bp.hot_count = ws->g->colx ? ws->g->hot_count : 0;
    bp.fr_hot = ws->b_fr_hot;
    bp.nz_v = ws->b_nz_v;
    bp.nz_ts = ws->b_nz_ts;
    bp.sources = ws->b_sources;
    bp.ctrl = ws->ctrl;
    bp.stat_nl = ws->stat_nl;
    bp.stat_el = ws->stat_el;
    bp.max_tiles = ws->b_max_tiles;
    bp.utiles = ws->b_utiles;
    bp.desc_cap = ws->b_desc_cap;
    bp.bvt = ws->b_bvt;
    bp.uv = ws->b_uv;
    bp.spin_ticks = kSpinTicks;
    return bp;
}

int32_t batch_pull_edges(const bfs_workspace_s* ws) {
    // pulling reads every row once; pushing costs up to four atomics per active edge
    return ws->batch_pull >= -1 ? (ws->batch_pull < 0 ? INT32_MAX : ws->batch_pull)
                                : (int32_t)std::min<int64_t>(ws->g->m / 8, INT32_MAX);
}

int batch_grid(const bfs_workspace_s* ws) {
    return ws->grid_opt > 0 ? std::min(ws->grid_opt, ws->b_grid_cap) : ws->b_grid_cap;
}

// Captures batch_levels levels of the batched loop on the workspace's own
// stream.  Done when the workspace is made or its launch shape changes,
// never while a run is in progress.
bfs_status_t capture_batch(bfs_workspace_s* ws) {
    if (ws->b_exec) (void)hipGraphExecDestroy(ws->b_exec);
    if (ws->b_graph) (void)hipGraphDestroy(ws->b_graph);
    ws->b_exec = nullptr;
    ws->b_graph = nullptr;
    const BatchParams bp = make_batch_params(ws);
    const int grid = batch_grid(ws);
    HIP_TRY(hipStreamBeginCapture(ws->own_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < ws->batch_levels; ++i) {
        hipError_t e = launch_batch_level(bp, grid, ws->own_stream);
        if (e != hipSuccess) {
            hipGraph_t gdead = nullptr;
            (void)hipStreamEndCapture(ws->own_stream, &gdead);
            if (gdead) (void)hipGraphDestroy(gdead);
            return fail(BFS_EHIP, "capturing the batched level loop: %s", hipGetErrorString(e));
        }
    }
    HIP_TRY(hipStreamEndCapture(ws->own_stream, &ws->b_graph));
    HIP_TRY(hipGraphInstantiate(&ws->b_exec, ws->b_graph, nullptr, nullptr, 0));
    return BFS_OK;
}

// Waits for the workspace's last run, so that its launch shape can change.
bfs_status_t quiesce(bfs_workspace_s* ws) {
    if (ws->has_run) HIP_TRY(hipEventSynchronize(ws->ev_done));
    return BFS_OK;
}

// The grain-dependent set-up (sub-tile starts over all edges) and the
// occupancy of the expansion kernel, then a new capture of the level loop.
bfs_status_t setup_batch(bfs_workspace_s* ws) {
    hipStream_t os = ws->own_stream;
    ws->b_grid_cap = batch_grid_capacity(ws->device, ws->b_bvt);
    if (ws->b_grid_cap <= 0) return fail(BFS_EHIP, "could not size the batched grid");
    ws->b_utiles = (int32_t)(((int64_t)ws->g->n + (int64_t)kBlock * ws->b_uv - 1) / ((int64_t)kBlock * ws->b_uv));
    const BatchParams bp = make_batch_params(ws);
    HIP_TRY(launch_batch_args(ws->b_args, BatchArgs{nullptr, 0, 0, batch_pull_edges(ws), 0}, os));
    HIP_TRY(launch_batch_setup(bp, ws->b_grid_cap, os));
    HIP_TRY(hipStreamSynchronize(os));
    return capture_batch(ws);
}

}  // namespace

// ---- scratch of the search that allocates nothing ---------------------------------------
// One fixed array per device, held from the library's first graph on that
// device until the process ends.  Host code never uses its name as an
// address: the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

struct StaticScratch {
    std::mutex mu;
    unsigned char* ptr[kMaxDevices] = {};  // device address of `scratch` on each device
    int grid_cap[kMaxDevices] = {};        // co-resident workgroups of the level loop there
    uint64_t last_uid[kMaxDevices] = {};   // graph of the last search that used it (0: none)
};
StaticScratch g_static;

// Looks up the device's copy of the scratch array (with that device current),
// once per device.
bfs_status_t static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(BFS_EHIP, "device %d beyond the library's %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_static.mu);
    if (g_static.ptr[device]) return BFS_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(BFS_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    const int cap = persistent_grid_capacity(device);
    if (cap <= 0) return fail(BFS_EHIP, "could not size the persistent grid on device %d", device);
    g_static.grid_cap[device] = cap;
    g_static.ptr[device] = static_cast<unsigned char*>(ptr);
    return BFS_OK;
}

// Lays the arrays of one single-source search of g out from base, each
// 256-byte aligned, in p's workspace fields (base == nullptr: sizes only).
// Returns the bytes used.
size_t carve_single(const bfs_graph_s* g, unsigned char* base, Params* p) {
    const size_t n = (size_t)g->n;
    const size_t T = (size_t)((std::max<int64_t>(g->m, g->n) + kGrain - 1) / kGrain + 2);
    const size_t W = (n + 31) / 32;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* q = base ? base + off : nullptr;
        off += (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
        return q;
    };
    p->bitmap = static_cast<uint32_t*>(take(W * 4));
    p->fbits[0] = static_cast<uint32_t*>(take(W * 4));
    p->fbits[1] = static_cast<uint32_t*>(take(W * 4));
    p->snap = static_cast<uint32_t*>(take(W * 4));
    p->hot[0] = p->hot[1] = nullptr;
    if (g->colx) {
        p->hot[0] = static_cast<uint32_t*>(take((size_t)g->hot_words * 4));
        p->hot[1] = static_cast<uint32_t*>(take((size_t)g->hot_words * 4));
    }
    p->owner = static_cast<int32_t*>(take(n * 4));
    for (int i = 0; i < 2; ++i) {
        p->f_rs[i] = static_cast<int32_t*>(take((n + 2) * 4));
        p->f_ex[i] = static_cast<int32_t*>(take((n + 2) * 4));
        p->f_v[i] = static_cast<int32_t*>(take((n + 2) * 4));
        p->tstart[i] = static_cast<int32_t*>(take(T * 4));
        p->desc[i] = static_cast<unsigned long long*>(take(T * 8));
    }
    p->cand_cap = default_cand(g->m, g->n);
    p->cand = static_cast<int32_t*>(take((size_t)p->cand_cap * 4));
    for (int i = 0; i < 2; ++i) {
        p->gv[i] = static_cast<int32_t*>(take((size_t)kGroupCap * 4));
        p->grs[i] = static_cast<int32_t*>(take((size_t)kGroupCap * 4));
        p->gd[i] = static_cast<int32_t*>(take((size_t)kGroupCap * 4));
    }
    p->cnt = static_cast<int32_t*>(take(2 * T * 4));
    p->ctrl = static_cast<Ctrl*>(take(sizeof(Ctrl)));
    p->xbar = static_cast<XBar*>(take(sizeof(XBar)));
    p->aux = static_cast<Aux*>(take(sizeof(Aux)));
    p->stat_nl = static_cast<int32_t*>(take((size_t)kStatCap * 4));
    p->stat_el = static_cast<int32_t*>(take((size_t)kStatCap * 4));
    p->stat_ts = static_cast<uint64_t*>(take(3 * (size_t)kStatCap * 8));
    p->max_tiles = (int32_t)T;
    return off;
}

}  // namespace

// Hot-vertex filter of a resident graph: number the (at most kHotBits) vertices
// of highest degree, ties by id, in id order (numbering them by degree packs the
// hubs' hot bits into a few words, which then cost the expansion more in atomic
// contention than the batched pull gains from the denser masks); each edge's
// entry of colx holds its target, or -1 - the target's hot number, and hot_vid
// maps hot numbers back to ids.
static bfs_status_t build_hot_filter(bfs_graph_s* g, const int32_t* host_offsets, hipStream_t s) {
    const int32_t n = g->n;
    std::vector<int32_t> ho;
    if (!host_offsets) {
        ho.resize((size_t)n + 1);
        HIP_TRY(hipMemcpy(ho.data(), g->offsets, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
        host_offsets = ho.data();
    }
    std::vector<int32_t> deg((size_t)n);
    int64_t nz = 0;
    for (int32_t v = 0; v < n; ++v) {
        deg[v] = host_offsets[v + 1] - host_offsets[v];
        nz += deg[v] > 0;
    }
    const int64_t K = std::min<int64_t>(kHotBits, nz);
    if (K == 0) return BFS_OK;
    // t = the K-th largest degree: every vertex above it is hot, then ties by id
    std::vector<int32_t> tmp(deg);
    std::nth_element(tmp.begin(), tmp.begin() + (K - 1), tmp.end(), std::greater<int32_t>());
    const int32_t t = std::max(tmp[K - 1], 1);
    tmp.clear();
    tmp.shrink_to_fit();
    std::vector<int32_t> hidx((size_t)n, -1), hvid;
    hvid.reserve((size_t)K);
    for (int32_t v = 0; v < n; ++v)
        if (deg[v] > t) {
            hidx[v] = (int32_t)hvid.size();
            hvid.push_back(v);
        }
    for (int32_t v = 0; v < n && (int64_t)hvid.size() < K; ++v)
        if (deg[v] == t) {
            hidx[v] = (int32_t)hvid.size();
            hvid.push_back(v);
        }
    const int32_t cnt = (int32_t)hvid.size();
    int32_t* d_hidx = nullptr;
    if (dalloc(&d_hidx, (size_t)n) != hipSuccess || dalloc(&g->colx, (size_t)g->m) != hipSuccess ||
        dalloc(&g->hot_vid, (size_t)cnt) != hipSuccess) {
        (void)hipFree(d_hidx);
        (void)hipFree(g->colx);
        (void)hipFree(g->hot_vid);
        g->colx = g->hot_vid = nullptr;
        return fail(BFS_ENOMEM, "device allocation of the hot-vertex filter failed");
    }
    hipError_t e = hipMemcpyAsync(d_hidx, hidx.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->hot_vid, hvid.data(), sizeof(int32_t) * (size_t)cnt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_hot_gather(g->cols, g->m, d_hidx, g->colx, n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_hidx);
    if (e != hipSuccess) return fail(BFS_EHIP, "building the hot-vertex filter: %s", hipGetErrorString(e));
    g->hot_count = cnt;
    g->hot_words = (cnt + 31) / 32;
    return BFS_OK;
}

extern "C" {

const char* bfs_last_error(void) { return g_last_error.c_str(); }

const char* bfs_status_str(bfs_status_t s) {
    switch (s) {
        case BFS_OK: return "ok";
        case BFS_EINVAL: return "invalid argument";
        case BFS_ERANGE: return "source or root out of range";
        case BFS_ENOMEM: return "out of memory";
        case BFS_EBADCSR: return "malformed CSR graph";
        case BFS_EHIP: return "HIP runtime error";
        case BFS_EOVERFLOW: return "batched level reached 255";
        case BFS_EBUSY: return "workspace busy on another stream";
        case BFS_EDEVICE: return "device-side failure";
        default: return "unknown status";
    }
}

bfs_status_t bfs_init(const int32_t* offsets, const int32_t* cols, int32_t n, int64_t m, uint32_t flags,
                      void* stream, bfs_graph_t* out) {
    if (!out) return fail(BFS_EINVAL, "null output handle");
    *out = nullptr;
    if (!offsets || (m > 0 && !cols)) return fail(BFS_EINVAL, "null CSR pointer");
    if (n < 0 || m < 0 || m > INT32_MAX) return fail(BFS_EINVAL, "n or m out of range");
    const bool host = flags & BFS_HOST_PTRS, dev = flags & BFS_DEVICE_PTRS;
    if (host == dev) return fail(BFS_EINVAL, "exactly one of BFS_HOST_PTRS / BFS_DEVICE_PTRS");
    if (flags & ~(BFS_HOST_PTRS | BFS_DEVICE_PTRS | BFS_VALIDATE | BFS_HOT_FILTER | BFS_LEAN | BFS_SORT_ROWS))
        return fail(BFS_EINVAL, "unknown flag");
    const bool sort_rows = flags & BFS_SORT_ROWS;
    if ((flags & BFS_HOT_FILTER) && (flags & BFS_LEAN)) return fail(BFS_EINVAL, "BFS_HOT_FILTER and BFS_LEAN together");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (flags & BFS_VALIDATE) {
        std::vector<int32_t> ho, hc;
        const int32_t* po = offsets;
        const int32_t* pc = cols;
        if (dev) {
            ho.resize((size_t)n + 1);
            hc.resize((size_t)std::max<int64_t>(m, 1));
            HIP_TRY(hipMemcpy(ho.data(), offsets, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
            if (m) HIP_TRY(hipMemcpy(hc.data(), cols, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost));
            po = ho.data();
            pc = hc.data();
        } else if (sort_rows) {
            hc.assign(cols, cols + m);
            pc = hc.data();
        }
        if (sort_rows) {
            // what the device sort will produce, checked here (offsets first, so that the rows exist)
            if (po[0] != 0 || (int64_t)po[n] != m) return fail(BFS_EBADCSR, "offsets do not span [0, m)");
            for (int32_t v = 0; v < n; ++v) {
                if (po[v + 1] < po[v]) return fail(BFS_EBADCSR, "offsets decrease at vertex %d", v);
                std::sort(hc.begin() + po[v], hc.begin() + po[v + 1]);
            }
        }
        bfs_status_t st = validate_csr(po, pc, n, m);
        if (st) return st;
    }
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    if (bfs_status_t st = static_scratch_setup(device)) return st;
    auto* g = new (std::nothrow) bfs_graph_s();
    if (!g) return fail(BFS_ENOMEM, "host allocation failed");
    static std::atomic<uint64_t> next_uid{1};
    g->uid = next_uid.fetch_add(1);
    g->device = device;
    g->n = n;
    g->m = m;
    if (dev) {
        g->offsets = const_cast<int32_t*>(offsets);
        g->cols = const_cast<int32_t*>(cols);
        g->owned = false;
    } else {
        if (dalloc(&g->offsets, (size_t)n + 1) != hipSuccess || dalloc(&g->cols, (size_t)m) != hipSuccess) {
            (void)hipFree(g->offsets);
            (void)hipFree(g->cols);
            delete g;
            return fail(BFS_ENOMEM, "device allocation of the CSR failed");
        }
        g->owned = true;
        HIP_TRY(hipMemcpyAsync(g->offsets, offsets, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice, s));
        if (m) HIP_TRY(hipMemcpyAsync(g->cols, cols, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (sort_rows && m > 0) {
        int32_t* sorted = nullptr;
        if (dalloc(&sorted, (size_t)m) != hipSuccess) {
            bfs_graph_free(g);
            return fail(BFS_ENOMEM, "device allocation of the sorted rows failed");
        }
        const hipError_t e = sort_rows_device(g->offsets, g->cols, sorted, n, m, s);
        if (e != hipSuccess) {
            (void)hipFree(sorted);
            bfs_graph_free(g);
            return fail(BFS_EHIP, "sorting the rows: %s", hipGetErrorString(e));
        }
        if (g->owned) (void)hipFree(g->cols);  // the unsorted upload
        g->cols = sorted;
        g->owned_cols = !g->owned;
    }
    const bool want_hot = !(flags & BFS_LEAN) && ((flags & BFS_HOT_FILTER) || m >= kHotMinEdges) && n > 0 && m > 0;
    if (want_hot) {
        bfs_status_t st = build_hot_filter(g, host ? offsets : nullptr, s);
        if (st) {
            bfs_graph_free(g);
            return st;
        }
    }
    *out = g;
    return BFS_OK;
}

bfs_status_t bfs_graph_free(bfs_graph_t g) {
    if (!g) return fail(BFS_EINVAL, "null graph");
    if (g->owned) {
        (void)hipFree(g->offsets);
        (void)hipFree(g->cols);
    } else if (g->owned_cols) {
        (void)hipFree(g->cols);
    }
    if (g->colx) (void)hipFree(g->colx);
    if (g->hot_vid) (void)hipFree(g->hot_vid);
    delete g;
    return BFS_OK;
}

int64_t bfs_graph_aux_bytes(bfs_graph_t g) {
    return g && g->colx ? (g->m + g->hot_count) * (int64_t)sizeof(int32_t) : 0;
}

bfs_status_t bfs_graph_info(bfs_graph_t g, int32_t* n, int64_t* m) {
    if (!g) return fail(BFS_EINVAL, "null graph");
    if (n) *n = g->n;
    if (m) *m = g->m;
    return BFS_OK;
}

static int64_t tiles_for(const bfs_graph_s* g) {
    const int64_t items = std::max<int64_t>(g->m, g->n);
    return (items + kGrain - 1) / kGrain + 2;
}

static int64_t batch_max_tiles(const bfs_graph_s* g) {
    const int64_t G = (int64_t)kBlock * kBVTMin;   // the finest grain
    return (g->m + G - 1) / G + 2;
}

static int64_t batch_desc_cap(const bfs_graph_s* g) {
    const int64_t a = ((int64_t)g->n + (int64_t)kBlock * kUVMin - 1) / ((int64_t)kBlock * kUVMin);
    const int64_t b = ((int64_t)g->n + kNzTile - 1) / kNzTile;
    return std::max<int64_t>(std::max(a, b), 1);
}

size_t bfs_workspace_bytes(bfs_graph_t g, int32_t max_sources) {
    if (!g || max_sources < 1 || max_sources > 256) return 0;
    const size_t n = (size_t)g->n, T = (size_t)tiles_for(g);
    size_t b = 0;
    b += 4 * ((n + 31) / 32) * 4;      // visited bitmap, frontier bits x2, dense-level snapshot
    if (g->colx) b += 2 * (size_t)g->hot_words * 4;  // hot-vertex bits x2
    b += n * 4;                        // owner
    b += 6 * (n + 2) * 4;              // frontier ids / row starts / degree sums, x2
    b += 2 * T * 4;                    // tstart x2
    b += (size_t)default_cand(g->m, g->n) * 4;  // private queues (default options; see bfs.h)
    b += 2 * T * 4;                    // counts, bottom-up edge totals
    b += 2 * T * 8;                    // descriptors
    b += 6 * (size_t)kGroupCap * 4;    // group levels' frontier entries x2
    b += sizeof(Ctrl) + sizeof(XBar) + sizeof(Aux) + 2 * (size_t)kStatCap * 4 + 3 * (size_t)kStatCap * 8 + n * 4;  // ctrl, barrier, stats, roots
    if (max_sources > 1) {
        const size_t BT = (size_t)batch_max_tiles(g), D = (size_t)batch_desc_cap(g);
        b += 3 * n * 32;               // frontier/next/visited masks
        b += 6 * (n + 2) * 4;          // active ids / row starts / degree sums, x2
        b += 3 * BT * 4;               // sub-tile starts x2, over all edges
        b += 2 * D * 8;                // update descriptors x2
        b += ((n + 31) / 32 + 1) * 4 + (n + 1) * 4 + 256 * 4 + sizeof(BatchArgs);  // active bits, nz list, sources
        if (g->colx) b += (size_t)g->hot_count * 32;  // hot vertices' frontier masks
    }
    return b;
}

bfs_status_t bfs_workspace_free(bfs_workspace_t ws) {
    if (!ws) return fail(BFS_EINVAL, "null workspace");
    (void)hipSetDevice(ws->device);
    if (ws->has_run) (void)hipEventSynchronize(ws->ev_done);
    if (ws->b_exec) (void)hipGraphExecDestroy(ws->b_exec);
    if (ws->b_graph) (void)hipGraphDestroy(ws->b_graph);
    for (void* q : {static_cast<void*>(ws->plain_fv[0]), static_cast<void*>(ws->plain_fv[1])})
        if (q) (void)hipFree(q);
    // the arena (and a grown queue array) go back on the workspace's own stream, behind its last use
    pool_free(ws->cand_grown, ws->cand_pooled, ws->own_stream);
    pool_free(ws->arena, ws->arena_pooled, ws->own_stream);
    stream_give(ws->device, ws->own_stream);
    pinned_ctrl_give(ws->h_ctrl);
    if (ws->ev_ready) (void)hipEventDestroy(ws->ev_ready);
    if (ws->ev_done) (void)hipEventDestroy(ws->ev_done);
    if (ws->ev0) (void)hipEventDestroy(ws->ev0);
    if (ws->ev1) (void)hipEventDestroy(ws->ev1);
    for (auto& pe : ws->prof_ev) {
        (void)hipEventDestroy(pe.first);
        (void)hipEventDestroy(pe.second);
    }
    delete ws;
    return BFS_OK;
}

bfs_status_t bfs_workspace_create(bfs_graph_t g, int32_t max_sources, bfs_workspace_t* out) {
    if (!out || !g) return fail(BFS_EINVAL, "null argument");
    *out = nullptr;
    if (max_sources < 1 || max_sources > 256) return fail(BFS_EINVAL, "max_sources must be in [1, 256]");
    auto* ws = new (std::nothrow) bfs_workspace_s();
    if (!ws) return fail(BFS_ENOMEM, "host allocation failed");
    ws->g = g;
    ws->device = g->device;
    ws->max_sources = max_sources;
    HIP_TRY(hipSetDevice(ws->device));
    const size_t n = (size_t)g->n;
    const int64_t T = tiles_for(g);
    ws->max_tiles = (int32_t)T;
    // everything is set up on the workspace's own stream (no device-wide synchronisation)
    if (stream_take(ws->device, &ws->own_stream) != hipSuccess) {
        bfs_workspace_free(ws);
        return fail(BFS_EHIP, "could not create the workspace stream");
    }
    // one arena: the bytes bfs_workspace_bytes counts, plus each slice's alignment
    const size_t want = bfs_workspace_bytes(g, max_sources) + 64 * kSliceAlign;
    bool okk = pool_alloc(ws->device, ws->own_stream, want, &ws->arena, &ws->arena_pooled) == hipSuccess;
    if (okk) ws->arena_bytes = want;
    auto A = [&](hipError_t e) { okk = okk && e == hipSuccess; };
    A(take(ws, &ws->bitmap, (n + 31) / 32));
    A(take(ws, &ws->fbits[0], (n + 31) / 32));
    A(take(ws, &ws->fbits[1], (n + 31) / 32));
    A(take(ws, &ws->snap, (n + 31) / 32));
    if (g->colx) {
        A(take(ws, &ws->hot[0], (size_t)g->hot_words));
        A(take(ws, &ws->hot[1], (size_t)g->hot_words));
    }
    A(take(ws, &ws->owner, n));
    for (int i = 0; i < 2; ++i) {
        A(take(ws, &ws->f_rs[i], n + 2));
        A(take(ws, &ws->f_ex[i], n + 2));
        A(take(ws, &ws->f_v[i], n + 2));
        A(take(ws, &ws->tstart[i], (size_t)T));
        A(take(ws, &ws->desc[i], (size_t)T));
        A(take(ws, &ws->gv[i], (size_t)kGroupCap));
        A(take(ws, &ws->grs[i], (size_t)kGroupCap));
        A(take(ws, &ws->gd[i], (size_t)kGroupCap));
    }
    ws->cand_cap = default_cand(g->m, g->n);
    A(take(ws, &ws->cand, (size_t)ws->cand_cap));
    A(take(ws, &ws->cnt, 2 * (size_t)T));    // queue lengths, then bottom-up edge totals
    A(take(ws, &ws->ctrl, 1));
    A(take(ws, &ws->xbar, 1));
    A(take(ws, &ws->aux, 1));
    A(take(ws, &ws->stat_nl, kStatCap));
    A(take(ws, &ws->stat_el, kStatCap));
    A(take(ws, &ws->stat_ts, 3 * (size_t)kStatCap));
    A(take(ws, &ws->roots, n));
    if (max_sources > 1) {
        ws->b_max_tiles = (int32_t)batch_max_tiles(g);
        ws->b_desc_cap = (int32_t)batch_desc_cap(g);
        A(take(ws, &ws->b_fr, n * 4));
        A(take(ws, &ws->b_nx, n * 4));
        A(take(ws, &ws->b_vis, n * 4));
        for (int i = 0; i < 2; ++i) {
            A(take(ws, &ws->b_act[i], n + 2));
            A(take(ws, &ws->b_act_rs[i], n + 2));
            A(take(ws, &ws->b_act_ex[i], n + 2));
            A(take(ws, &ws->b_tstart[i], (size_t)ws->b_max_tiles));
            A(take(ws, &ws->b_desc[i], (size_t)ws->b_desc_cap));
        }
        A(take(ws, &ws->b_act_bits, (n + 31) / 32 + 1));
        if (g->colx) A(take(ws, &ws->b_fr_hot, (size_t)g->hot_count * 4));
        A(take(ws, &ws->b_nz_v, n + 1));
        A(take(ws, &ws->b_nz_ts, (size_t)ws->b_max_tiles));
        A(take(ws, &ws->b_sources, 256));
        A(take(ws, &ws->b_args, 1));
    }
    if (okk && pinned_ctrl_take(&ws->h_ctrl) != hipSuccess) okk = false;
    if (okk && (hipEventCreate(&ws->ev_done) != hipSuccess || hipEventCreate(&ws->ev0) != hipSuccess ||
                hipEventCreate(&ws->ev1) != hipSuccess ||
                hipEventCreateWithFlags(&ws->ev_ready, hipEventDisableTiming) != hipSuccess))
        okk = false;
    if (!okk) {
        bfs_workspace_free(ws);
        return fail(BFS_ENOMEM, "workspace allocation failed (%zu bytes requested)", bfs_workspace_bytes(g, max_sources));
    }
    ws->grid_cap = persistent_grid_capacity(ws->device);
    if (ws->grid_cap <= 0) {
        bfs_workspace_free(ws);
        return fail(BFS_EHIP, "could not size the persistent grid");
    }
    // defined contents everywhere, so no stale or never-written entry can hold an out-of-range index
    hipStream_t os = ws->own_stream;
    bool zok = hipMemsetAsync(ws->cnt, 0, sizeof(int32_t) * 2 * (size_t)T, os) == hipSuccess &&
               hipMemsetAsync(ws->cand, 0, sizeof(int32_t) * (size_t)ws->cand_cap, os) == hipSuccess &&
               hipMemsetAsync(ws->owner, 0xff, sizeof(int32_t) * n, os) == hipSuccess;
    for (int i = 0; i < 2 && zok; ++i)
        zok = hipMemsetAsync(ws->tstart[i], 0, sizeof(int32_t) * (size_t)T, os) == hipSuccess &&
              hipMemsetAsync(ws->f_rs[i], 0, sizeof(int32_t) * (n + 2), os) == hipSuccess &&
              hipMemsetAsync(ws->f_ex[i], 0, sizeof(int32_t) * (n + 2), os) == hipSuccess &&
              hipMemsetAsync(ws->f_v[i], 0, sizeof(int32_t) * (n + 2), os) == hipSuccess &&
              hipMemsetAsync(ws->desc[i], 0, sizeof(unsigned long long) * (size_t)T, os) == hipSuccess;
    // the clears stay queued on the workspace's stream: a synchronisation here would also wait
    // for whatever shares its hardware queue; runs on other streams wait for ev_ready instead
    if (!zok || hipMemsetAsync(ws->ctrl, 0, sizeof(Ctrl), os) != hipSuccess ||
        hipEventRecord(ws->ev_ready, os) != hipSuccess) {
        bfs_workspace_free(ws);
        return fail(BFS_EHIP, "hipMemset failed");
    }
    ws->init_pending = true;
    if (max_sources > 1) {
        bfs_status_t cst = setup_batch(ws);
        if (cst) {
            bfs_workspace_free(ws);
            return cst;
        }
    }
    *out = ws;
    return BFS_OK;
}

bfs_status_t bfs_workspace_set_option(bfs_workspace_t ws, int32_t option, int64_t value) {
    if (!ws) return fail(BFS_EINVAL, "null workspace");
    switch (option) {
        case BFS_OPT_MODE:
            if (value < BFS_MODE_AUTO || value > BFS_MODE_DIRECTION) return fail(BFS_EINVAL, "bad mode");
            ws->mode = (int32_t)value;
            return BFS_OK;
        case BFS_OPT_SMALL_EDGES:
            if (value < 0 || value > INT32_MAX) return fail(BFS_EINVAL, "bad small-edge threshold");
            ws->small_edges = (int32_t)value;
            return BFS_OK;
        case BFS_OPT_GRID: {
            if (value < 0 || value > INT32_MAX) return fail(BFS_EINVAL, "bad grid");
            if (bfs_status_t q = quiesce(ws)) return q;
            ws->grid_opt = (int32_t)value;
            return ws->b_exec ? capture_batch(ws) : BFS_OK;
        }
        case BFS_OPT_BU_ALPHA:
            if (value < 1 || value > (1 << 20)) return fail(BFS_EINVAL, "alpha must be in [1, 2^20]");
            ws->bu_alpha = (int32_t)value;
            return BFS_OK;
        case BFS_OPT_BU_BETA:
            if (value < 1 || value > (1 << 20)) return fail(BFS_EINVAL, "beta must be in [1, 2^20]");
            ws->bu_beta = (int32_t)value;
            return BFS_OK;
        case BFS_OPT_PROFILE:
            ws->profile = value != 0;
            return BFS_OK;
        case BFS_OPT_PUSH_EDGES:
            if (value < 0 || value > INT32_MAX) return fail(BFS_EINVAL, "bad push threshold");
            ws->push_edges = (int32_t)value;
            return BFS_OK;
        case BFS_OPT_DENSE_EDGES:
            if (value < 0 || value > INT32_MAX) return fail(BFS_EINVAL, "bad dense threshold");
            ws->dense_edges = (int32_t)value;
            return BFS_OK;
        case BFS_OPT_HOST_STATUS:
            if (value != 0 && value != 1) return fail(BFS_EINVAL, "BFS_OPT_HOST_STATUS is 0 or 1");
            ws->host_status_copy = value != 0;
            return BFS_OK;
        case BFS_OPT_BATCH_REPLAYS:
            if (value < -1 || value > 256) return fail(BFS_EINVAL, "replays per batched run must be in [-1, 256]");
            ws->batch_replays = (int32_t)value;
            return BFS_OK;
        case BFS_OPT_BATCH_LEVELS: {
            if (value < 1 || value > 256) return fail(BFS_EINVAL, "levels per replay must be in [1, 256]");
            if (bfs_status_t q = quiesce(ws)) return q;
            ws->batch_levels = (int32_t)value;
            return ws->b_exec ? capture_batch(ws) : BFS_OK;
        }
        case BFS_OPT_BATCH_GRAIN: {
            if (value != 512 && value != 1024 && value != 2048)
                return fail(BFS_EINVAL, "batched grain must be 512, 1024 or 2048 edges");
            if (ws->max_sources < 2) return fail(BFS_EINVAL, "the workspace has no batched buffers");
            if (bfs_status_t q = quiesce(ws)) return q;
            ws->b_bvt = (int32_t)(value / kBlock);
            return setup_batch(ws);
        }
        case BFS_OPT_BATCH_TILE: {
            if (value != 1024 && value != 2048 && value != 4096)
                return fail(BFS_EINVAL, "batched update tile must be 1024, 2048 or 4096 vertices");
            if (ws->max_sources < 2) return fail(BFS_EINVAL, "the workspace has no batched buffers");
            if (bfs_status_t q = quiesce(ws)) return q;
            ws->b_uv = (int32_t)(value / kBlock);
            return setup_batch(ws);
        }
        case BFS_OPT_GROUP:
            if (value < 0 || value > kGroupLimit) return fail(BFS_EINVAL, "group must be in [0, %d]", kGroupLimit);
            ws->group = value == 0 ? kGroupMax : (int32_t)value;
            return BFS_OK;
        case BFS_OPT_SPLIT:
            if (value != 0 && value != 1) return fail(BFS_EINVAL, "split must be 0 (scatter) or 1 (binary search)");
            ws->split_search = (int32_t)value;
            return BFS_OK;
        case BFS_OPT_BATCH_PULL:
            if (value < -1 || value > INT32_MAX) return fail(BFS_EINVAL, "bad pull threshold");
            ws->batch_pull = (int32_t)value;
            return BFS_OK;
        default:
            return fail(BFS_EINVAL, "unknown option %d", option);
    }
}

bfs_status_t bfs_run(bfs_workspace_t ws, int32_t source, int32_t* level, int32_t* parent, void* stream) {
    return run_common(ws, nullptr, 0, source, level, parent, stream);
}

bfs_status_t bfs_run_multiroot(bfs_workspace_t ws, const int32_t* roots, int32_t k, int32_t* level,
                               int32_t* parent, void* stream) {
    if (!ws) return fail(BFS_EINVAL, "null workspace");
    if (!roots || k < 1 || k > ws->g->n) return fail(BFS_EINVAL, "need 1 <= k <= n roots");
    return run_common(ws, roots, k, 0, level, parent, stream);
}

bfs_status_t bfs_run_noalloc(bfs_graph_t g, int32_t source, int32_t* level, int32_t* parent, int32_t* status,
                             void* stream) {
    if (!g) return fail(BFS_EINVAL, "null graph");
    if (!level) return fail(BFS_EINVAL, "null level array");
    if (source < 0 || source >= g->n) return fail(BFS_ERANGE, "source %d outside [0, %d)", source, g->n);
    Params p{};
    const size_t need = carve_single(g, nullptr, &p);
    if (need > kStaticScratchBytes)
        return fail(BFS_ENOMEM, "the graph (n = %d, m = %lld) needs %zu bytes of search scratch; the static scratch "
                    "holds %zu", g->n, (long long)g->m, need, kStaticScratchBytes);
    if (g->device < 0 || g->device >= kMaxDevices) return fail(BFS_EHIP, "device %d beyond the library's", g->device);
    unsigned char* base = nullptr;
    int cap = 0;
    bool scrub = false;
    {
        std::lock_guard<std::mutex> lk(g_static.mu);
        base = g_static.ptr[g->device];
        cap = g_static.grid_cap[g->device];
        scrub = g_static.last_uid[g->device] != g->uid;
        g_static.last_uid[g->device] = g->uid;
    }
    if (!base) return fail(BFS_EHIP, "no static scratch on device %d", g->device);
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    carve_single(g, base, &p);
    // the defaults of BFS_MODE_AUTO, as in a fresh workspace
    p.offsets = g->offsets;
    p.cols = g->cols;
    p.colx = g->colx;
    p.hot_vid = g->hot_vid;
    p.hot_count = g->colx ? g->hot_count : 0;
    p.hot_words = g->colx ? g->hot_words : 0;
    p.n = g->n;
    p.m = g->m;
    p.level = level;
    p.parent = parent;
    p.roots = nullptr;
    p.single_root = source;
    p.nroots = 1;
    p.small_edges = kDefaultSmallEdges;
    p.group = kGroupMax;
    p.push_edges = (int32_t)std::min<int64_t>(g->m / kLevelSplit, INT32_MAX);
    p.dense_edges = (int32_t)std::min<int64_t>(std::max<int64_t>(g->m / kLevelSplit, 1), INT32_MAX);
    p.bu_alpha = 14;
    p.bu_beta = 24;
    p.fb_pull = parent != nullptr;
    p.spin_ticks = kSpinTicks;
    const int grid = default_grid(cap, g->m);
    if (scrub) HIP_TRY(launch_scrub(p, s));
    HIP_TRY(launch_prep(p, 1, parent != nullptr, s));
    HIP_TRY(launch_persistent(p, grid, s));
    if (status) HIP_TRY(launch_status(p.ctrl, status, s));
    return BFS_OK;
}

bfs_status_t bfs_sync(bfs_workspace_t ws) {
    if (!ws) return fail(BFS_EINVAL, "null workspace");
    if (!ws->has_run) return BFS_OK;
    HIP_TRY(hipSetDevice(ws->device));
    HIP_TRY(hipEventSynchronize(ws->ev_done));
    if (ws->host_status != BFS_OK) return ws->host_status;
    // on the workspace's own non-blocking stream: waits for nothing else in flight on the device
    HIP_TRY(hipMemcpyAsync(ws->h_ctrl, ws->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, ws->own_stream));
    HIP_TRY(hipStreamSynchronize(ws->own_stream));
    if (ws->last_batch && !ws->h_ctrl->error && !ws->h_ctrl->batch_overflow) {
        const int32_t lv = ws->h_ctrl->levels;
        ws->b_seen = std::max(ws->b_seen, lv);
        int32_t d = ws->g->batch_depth.load(std::memory_order_relaxed);
        while (d < lv && !ws->g->batch_depth.compare_exchange_weak(d, lv, std::memory_order_relaxed)) {
        }
    }
    if (ws->h_ctrl->error)
        return fail(BFS_EDEVICE, "device-side failure (code %d: %s)", ws->h_ctrl->error,
                    ws->h_ctrl->error == -9 ? "malformed frontier" : "a wait timed out");
    if (ws->h_ctrl->batch_overflow) return fail(BFS_EOVERFLOW, "batched search reached level 255");
    return BFS_OK;
}

bfs_status_t bfs_run_status(bfs_workspace_t ws, int32_t* status) {
    if (!ws || !status) return fail(BFS_EINVAL, "null argument");
    if (!ws->has_run) {
        *status = BFS_OK;
        return BFS_OK;
    }
    if (ws->host_status != BFS_OK) {
        *status = ws->host_status;
        return BFS_OK;
    }
    if (!ws->status_copied)
        return fail(BFS_EINVAL, "the last run was batched or launched without BFS_OPT_HOST_STATUS");
    HIP_TRY(hipSetDevice(ws->device));
    const hipError_t q = hipEventQuery(ws->ev_done);
    if (q == hipErrorNotReady) return fail(BFS_EBUSY, "the run is still in flight");
    if (q != hipSuccess) return fail(BFS_EHIP, "hipEventQuery: %s", hipGetErrorString(q));
    const int32_t e = __atomic_load_n(&ws->h_ctrl->error, __ATOMIC_ACQUIRE);
    *status = e ? BFS_EDEVICE : BFS_OK;
    return BFS_OK;
}

bfs_status_t bfs_last_stats(bfs_workspace_t ws, bfs_stats_t* out) {
    if (!ws || !out) return fail(BFS_EINVAL, "null argument");
    bfs_status_t st = bfs_sync(ws);
    std::memset(out, 0, sizeof(*out));
    out->status = st;
    out->mode = ws->last_mode;
    out->grid = ws->last_grid;
    out->kernel_ms = -1.0;
    if (!ws->has_run) return BFS_OK;
    if (ws->profiled && ws->prof_used > 0) {
        float ms = 0;
        const auto& pe = ws->prof_ev[ws->prof_used - 1];
        if (hipEventElapsedTime(&ms, pe.first, pe.second) == hipSuccess) out->kernel_ms = ms;
    }
    if (ws->host_stats) {
        out->levels = (int32_t)ws->h_nl.size();
        for (size_t i = 0; i < ws->h_nl.size(); ++i) {
            out->reached += ws->h_nl[i];
            out->edges += ws->h_el[i] > 0 ? ws->h_el[i] : 0;
        }
        return BFS_OK;
    }
    out->levels = ws->h_ctrl->levels;
    out->small_levels = ws->h_ctrl->small_levels;
    out->bottom_up_levels = ws->h_ctrl->bu_levels;
    const int cnt = std::min(out->levels, kStatCap);
    out->stats_truncated = out->levels > kStatCap;
    std::vector<int32_t> a((size_t)std::max(cnt, 1)), b((size_t)std::max(cnt, 1));
    if (cnt > 0) {
        HIP_TRY(hipMemcpy(a.data(), ws->stat_nl, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(b.data(), ws->stat_el, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
    }
    for (int i = 0; i < cnt; ++i) {
        out->reached += a[i];
        out->edges += b[i];
    }
    return BFS_OK;
}

bfs_status_t bfs_last_level_stats(bfs_workspace_t ws, int32_t cap, int64_t* n_l, int64_t* e_l, int32_t* count) {
    if (!ws || !count || cap < 0 || (cap > 0 && (!n_l || !e_l))) return fail(BFS_EINVAL, "bad argument");
    bfs_stats_t s;
    bfs_status_t st = bfs_last_stats(ws, &s);
    if (st) return st;
    if (ws->host_stats) {
        const int c = std::min<int>(cap, (int)ws->h_nl.size());
        for (int i = 0; i < c; ++i) {
            n_l[i] = ws->h_nl[i];
            e_l[i] = ws->h_el[i];
        }
        *count = c;
        return BFS_OK;
    }
    const int c = std::min(std::min(cap, s.levels), kStatCap);
    std::vector<int32_t> a((size_t)std::max(c, 1)), b((size_t)std::max(c, 1));
    if (c > 0) {
        HIP_TRY(hipMemcpy(a.data(), ws->stat_nl, sizeof(int32_t) * c, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(b.data(), ws->stat_el, sizeof(int32_t) * c, hipMemcpyDeviceToHost));
    }
    for (int i = 0; i < c; ++i) {
        n_l[i] = a[i];
        e_l[i] = b[i];
    }
    *count = c;
    return BFS_OK;
}

bfs_status_t bfs_kernel_times(bfs_workspace_t ws, int32_t cap, double* ms, int32_t* count) {
    if (!ws || !count || cap < 0 || (cap > 0 && !ms)) return fail(BFS_EINVAL, "bad argument");
    HIP_TRY(hipSetDevice(ws->device));
    int32_t c = 0;
    for (size_t i = 0; i < ws->prof_used; ++i) {
        const auto& pe = ws->prof_ev[i];
        HIP_TRY(hipEventSynchronize(pe.second));
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, pe.first, pe.second));
        if (c < cap) ms[c++] = t;
    }
    ws->prof_used = 0;
    *count = c;
    return BFS_OK;
}

bfs_status_t bfs_last_level_times(bfs_workspace_t ws, int32_t cap, double* expand_us, double* compact_us,
                                  int32_t* count) {
    if (!ws || !count || cap < 0 || (cap > 0 && (!expand_us || !compact_us))) return fail(BFS_EINVAL, "bad argument");
    bfs_stats_t s;
    bfs_status_t st = bfs_last_stats(ws, &s);
    if (st) return st;
    *count = 0;
    if (ws->host_stats) return BFS_OK;  // per-level launches are not timed on the device
    const int c = std::min(std::min(cap, s.levels), kStatCap);
    if (c <= 0) return BFS_OK;
    std::vector<uint64_t> ts(3 * (size_t)c);
    HIP_TRY(hipMemcpy(ts.data(), ws->stat_ts, sizeof(uint64_t) * ts.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < c; ++i) {
        const double t0 = (double)ts[3 * i], t1 = (double)ts[3 * i + 1], t2 = (double)ts[3 * i + 2];
        expand_us[i] = (t1 - t0) * 0.01;  // s_memrealtime runs at 100 MHz
        compact_us[i] = (t2 - t1) * 0.01;
    }
    *count = c;
    return BFS_OK;
}

int32_t bfs_prim_grain(void) { return kGrain; }

int32_t bfs_workspace_grid_capacity(bfs_workspace_t ws) { return ws ? ws->grid_cap : 0; }

bfs_status_t bfs_workspace_set_spin_ticks(bfs_workspace_t ws, uint64_t ticks) {
    if (!ws) return fail(BFS_EINVAL, "null workspace");
    ws->spin_ticks = ticks;
    return BFS_OK;
}

bfs_status_t bfs_prim_compact(const int32_t* offsets, int32_t n, const int32_t* owner, const int32_t* cand,
                              const int32_t* cnt, int32_t ntiles, int32_t* out_v, int32_t* out_rs, int32_t* out_ex,
                              int32_t* out_tstart, int32_t tstart_cap, int32_t* totals, void* stream) {
    if (!offsets || !owner || (ntiles > 0 && (!cand || !cnt)) || !out_v || !out_rs || !out_ex || !out_tstart ||
        !totals || n < 0 || ntiles < 0 || tstart_cap < 0)
        return fail(BFS_EINVAL, "bad argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned long long* desc = nullptr;
    Ctrl* ctrl = nullptr;
    uint32_t* bitmap = nullptr;
    HIP_TRY(dalloc(&desc, (size_t)std::max(ntiles, 1)));
    HIP_TRY(dalloc(&ctrl, 1));
    HIP_TRY(dalloc(&bitmap, ((size_t)n + 31) / 32));
    HIP_TRY(hipMemsetAsync(ctrl, 0, sizeof(Ctrl), s));
    HIP_TRY(hipMemsetAsync(bitmap, 0, std::max<size_t>(((size_t)n + 31) / 32, 1) * 4, s));
    hipError_t e = launch_prim_compact(offsets, n, owner, cand, cnt, ntiles, out_v, out_rs, out_ex, out_tstart,
                                       tstart_cap, totals, desc, ctrl, bitmap, s);
    hipError_t e2 = hipStreamSynchronize(s);
    Ctrl hc;
    hipError_t e3 = hipMemcpy(&hc, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
    (void)hipFree(desc);
    (void)hipFree(ctrl);
    (void)hipFree(bitmap);
    if (e != hipSuccess) return fail(BFS_EHIP, "launch: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(BFS_EHIP, "sync: %s", hipGetErrorString(e2));
    if (e3 != hipSuccess) return fail(BFS_EHIP, "copy: %s", hipGetErrorString(e3));
    if (hc.error) return fail(BFS_EDEVICE, "device wait timed out");
    return BFS_OK;
}

bfs_status_t bfs_run_batch(bfs_workspace_t ws, const int32_t* sources, int32_t k, uint8_t* level, void* stream) {
    if (!ws) return fail(BFS_EINVAL, "null workspace");
    if (!sources || !level) return fail(BFS_EINVAL, "null sources or level array");
    if (k < 1 || k > ws->max_sources)
        return fail(BFS_EINVAL, "k = %d outside [1, %d] (the workspace's max_sources)", k, ws->max_sources);
    if (!ws->b_fr) return fail(BFS_EINVAL, "workspace was created for single-source runs (max_sources = 1)");
    if (reinterpret_cast<uintptr_t>(level) % 4 != 0) return fail(BFS_EINVAL, "level array must be 4-byte aligned");
    for (int32_t j = 0; j < k; ++j)
        if (sources[j] < 0 || sources[j] >= ws->g->n)
            return fail(BFS_ERANGE, "source %d = %d outside [0, %d)", j, sources[j], ws->g->n);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    bfs_status_t st = check_busy(ws, s);
    if (st) return st;
    HIP_TRY(hipSetDevice(ws->device));
    if ((st = wait_ready(ws, s))) return st;
    ws->host_stats = false;
    ws->profiled = false;
    ws->last_mode = BFS_MODE_AUTO;
    ws->host_status = BFS_OK;
    HIP_TRY(hipMemcpyAsync(ws->b_sources, sources, sizeof(int32_t) * (size_t)k, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_batch_args(ws->b_args, BatchArgs{level, k, (k + 63) / 64, batch_pull_edges(ws), 0}, s));
    const BatchParams bp = make_batch_params(ws);
    const int grid = batch_grid(ws);
    std::pair<hipEvent_t, hipEvent_t>* pe = nullptr;
    if (ws->profile) {
        st = profile_slot(ws, &pe);
        if (st) return st;
        HIP_TRY(hipEventRecord(pe->first, s));
    }
    HIP_TRY(launch_batch_start(bp, s));
    // Replays of the captured levels, as many as the deepest completed run of this workspace,
    // or else of any workspace on the graph, needed (32 levels before the first), then one
    // workgroup that finishes whatever levels are left: the call never waits for the device,
    // and the search is complete in stream order.  Levels after the stop cost a replay's
    // launches, not its work.
    const int32_t seen = std::max(ws->b_seen, ws->g->batch_depth.load(std::memory_order_relaxed));
    const int depth = seen > 0 ? seen : 32;
    const int replays = ws->batch_replays >= 0 ? ws->batch_replays
                                               : (depth + ws->batch_levels - 1) / ws->batch_levels;
    for (int r = 0; r < replays; ++r) HIP_TRY(hipGraphLaunch(ws->b_exec, s));
    HIP_TRY(launch_batch_finish(bp, s));
    if (pe) {
        HIP_TRY(hipEventRecord(pe->second, s));
        ws->profiled = true;
    }
    ws->last_grid = grid;
    HIP_TRY(hipEventRecord(ws->ev_done, s));
    ws->last_stream = s;
    ws->has_run = true;
    ws->last_batch = true;
    ws->status_copied = false;
    return BFS_OK;
}

}  // extern "C"

// ---- autotuning ---------------------------------------------------------------------------

namespace {

void current_tuning(const bfs_workspace_s* ws, bfs_tune_t* t) {
    std::memset(t, 0, sizeof(*t));
    t->batch_grain = kBlock * ws->b_bvt;
    t->batch_tile = kBlock * ws->b_uv;
    t->batch_levels = ws->batch_levels;
    t->batch_pull = ws->batch_pull >= -1 ? ws->batch_pull : batch_pull_edges(ws);
    t->grid = ws->grid_opt;
    t->small_edges = ws->small_edges;
    t->push_edges = push_edges_of(ws);
    t->dense_edges = dense_edges_of(ws);
}

// Timed passes over the tuning sample with the workspace's current settings.
struct TuneSample {
    bfs_workspace_s* ws;
    const int32_t* sources;
    int32_t k;
    bool batch;
    uint8_t* out8;
    int32_t* lv;
    int32_t* par;
    int32_t trials = 0;

    double pass() {
        const auto t0 = std::chrono::steady_clock::now();
        if (batch) {
            if (bfs_run_batch(ws, sources, k, out8, ws->own_stream) != BFS_OK) return INFINITY;
        } else {
            for (int32_t j = 0; j < k; ++j)
                if (bfs_run(ws, sources[j], lv, par, ws->own_stream) != BFS_OK) return INFINITY;
        }
        if (bfs_sync(ws) != BFS_OK) return INFINITY;
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    // one untimed pass, then the median of three
    double measure() {
        ++trials;
        if (!std::isfinite(pass())) return INFINITY;
        double t[3];
        for (double& x : t) x = pass();
        std::sort(t, t + 3);
        return t[1];
    }
};

// Tries every value of one option (or pair of options) and keeps the fastest.
template <typename Apply>
bfs_status_t descend(TuneSample& smp, double* best, const std::vector<std::pair<int64_t, int64_t>>& cands,
                     std::pair<int64_t, int64_t> keep, Apply apply) {
    std::pair<int64_t, int64_t> arg = keep;
    for (const auto& c : cands) {
        if (c == keep) continue;
        if (bfs_status_t st = apply(c)) return st;
        const double t = smp.measure();
        if (t < *best) {
            *best = t;
            arg = c;
        }
    }
    return apply(arg);
}

}  // namespace

extern "C" {

bfs_status_t bfs_workspace_get_tuning(bfs_workspace_t ws, bfs_tune_t* out) {
    if (!ws || !out) return fail(BFS_EINVAL, "null argument");
    current_tuning(ws, out);
    return BFS_OK;
}

bfs_status_t bfs_autotune(bfs_workspace_t ws, const int32_t* sources, int32_t k, uint32_t what, bfs_tune_t* out) {
    if (!ws || !sources) return fail(BFS_EINVAL, "null argument");
    if (what != BFS_TUNE_BATCH && what != BFS_TUNE_SINGLE) return fail(BFS_EINVAL, "tune BATCH or SINGLE, one at a time");
    const bool batch = what == BFS_TUNE_BATCH;
    if (batch && (k < 2 || k > ws->max_sources || !ws->b_fr))
        return fail(BFS_EINVAL, "batched tuning needs 2 <= k <= max_sources (%d) sources", ws->max_sources);
    if (!batch && (k < 1 || k > 64)) return fail(BFS_EINVAL, "single-source tuning takes 1 to 64 sources");
    const bfs_graph_s* g = ws->g;
    for (int32_t j = 0; j < k; ++j)
        if (sources[j] < 0 || sources[j] >= g->n) return fail(BFS_ERANGE, "source %d = %d outside [0, %d)", j, sources[j], g->n);
    if (bfs_status_t q = quiesce(ws)) return q;
    HIP_TRY(hipSetDevice(ws->device));
    TuneSample smp{ws, sources, k, batch, nullptr, nullptr, nullptr};
    bool ok = batch ? dalloc(&smp.out8, (size_t)g->n * (size_t)k) == hipSuccess
                    : dalloc(&smp.lv, (size_t)g->n) == hipSuccess && dalloc(&smp.par, (size_t)g->n) == hipSuccess;
    auto release = [&] {
        if (smp.out8) (void)hipFree(smp.out8);
        if (smp.lv) (void)hipFree(smp.lv);
        if (smp.par) (void)hipFree(smp.par);
    };
    if (!ok) {
        release();
        return fail(BFS_ENOMEM, "tuning output arrays");
    }
    const int32_t saved_mode = ws->mode, saved_profile = ws->profile;
    ws->mode = BFS_MODE_AUTO;
    ws->profile = 0;
    bfs_tune_t start;
    current_tuning(ws, &start);
    double best = smp.measure();
    const double t_default = best;
    bfs_status_t st = std::isfinite(best) ? BFS_OK : fail(BFS_EDEVICE, "the starting configuration failed: %s",
                                                          bfs_last_error());
    const int64_t m = g->m;
    using P = std::pair<int64_t, int64_t>;
    if (!st && batch) {
        std::vector<P> shapes;
        for (int64_t gr : {512, 1024, 2048})
            for (int64_t ti : {1024, 2048, 4096}) shapes.push_back({gr, ti});
        st = descend(smp, &best, shapes, P{start.batch_grain, start.batch_tile}, [&](P c) {
            bfs_status_t e = bfs_workspace_set_option(ws, BFS_OPT_BATCH_GRAIN, c.first);
            return e ? e : bfs_workspace_set_option(ws, BFS_OPT_BATCH_TILE, c.second);
        });
        std::vector<P> pulls;
        for (int64_t d : {32, 16, 8, 4, 2}) pulls.push_back({std::min<int64_t>(m / d, INT32_MAX), 0});
        pulls.push_back({-1, 0});
        if (!st)
            st = descend(smp, &best, pulls, P{start.batch_pull, 0},
                         [&](P c) { return bfs_workspace_set_option(ws, BFS_OPT_BATCH_PULL, c.first); });
        std::vector<P> reps;
        for (int64_t r : {2, 4, 8, 16}) reps.push_back({r, 0});
        if (!st)
            st = descend(smp, &best, reps, P{start.batch_levels, 0},
                         [&](P c) { return bfs_workspace_set_option(ws, BFS_OPT_BATCH_LEVELS, c.first); });
    } else if (!st) {
        const int64_t cap = ws->grid_cap;
        std::vector<P> grids{{0, 0}};
        for (int64_t d : {1, 2, 4, 8}) grids.push_back({std::max<int64_t>(cap / d, 1), 0});
        st = descend(smp, &best, grids, P{start.grid, 0},
                     [&](P c) { return bfs_workspace_set_option(ws, BFS_OPT_GRID, c.first); });
        std::vector<P> smalls;
        for (int64_t e : {0, 2048, 4096, 8192, 16384}) smalls.push_back({e, 0});
        if (!st)
            st = descend(smp, &best, smalls, P{start.small_edges, 0},
                         [&](P c) { return bfs_workspace_set_option(ws, BFS_OPT_SMALL_EDGES, c.first); });
        // push and dense thresholds move together: a level above the split pulls its
        // parents and keeps its new vertices as bits (or, last, never as bits)
        std::vector<P> splits;
        for (int64_t d : {48, 32, 24, 16, 12, 8}) {
            const int64_t e = std::min<int64_t>(std::max<int64_t>(m / d, 1), INT32_MAX);
            splits.push_back({e, e});
        }
        splits.push_back({std::min<int64_t>(m / kLevelSplit, INT32_MAX), 0});
        if (!st)
            st = descend(smp, &best, splits, P{start.push_edges, start.dense_edges}, [&](P c) {
                bfs_status_t e = bfs_workspace_set_option(ws, BFS_OPT_PUSH_EDGES, c.first);
                return e ? e : bfs_workspace_set_option(ws, BFS_OPT_DENSE_EDGES, c.second);
            });
    }
    ws->mode = saved_mode;
    ws->profile = saved_profile;
    if (bfs_status_t q = quiesce(ws); q && !st) st = q;
    release();
    if (out) {
        current_tuning(ws, out);
        out->trials = smp.trials;
        out->default_ms = t_default;
        out->best_ms = best;
    }
    return st;
}

}  // extern "C"
