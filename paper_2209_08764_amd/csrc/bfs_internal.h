// Internal declarations shared by the kernels and the C-ABI layer of libbfs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s3bfs {

// ---- launch geometry -------------------------------------------------------------------
constexpr int kBlock = 512;               // threads per workgroup of the level loop
constexpr int kWaves = kBlock / 64;       // wave64
constexpr int kVT = 4;                    // edges per thread in one sub-tile
constexpr int kGrain = kBlock * kVT;      // edges per sub-tile (the share granularity), 2048
constexpr int kSlice = kGrain + 1;        // frontier entries a sub-tile can touch
constexpr int kPre = (kSlice + kBlock - 1) / kBlock;  // slice entries each thread prefetches
constexpr int kVTS = 8;                   // edges (or staged entries) per thread per round, group levels
constexpr int kSmallN = 4096;             // frontier capacity of group levels (staged in LDS)
constexpr int kGroupCap = 16384;          // most edges a group level scans (and entries it appends)
constexpr int kGroupMax = 48;             // default workgroups of the group
constexpr int kGroupLimit = 64;           // most workgroups a group may have
constexpr int kStatCap = 1 << 16;         // per-level statistics kept
constexpr int kDefaultSmallEdges = kGroupCap;
constexpr int kPullScan = 32;             // neighbours a lane tests before a row goes to the whole workgroup

// Hot-vertex filter: the kHotBits vertices of highest degree carry a number
// in [0, kHotBits), and large levels keep their visited bits in LDS.
constexpr int kHotWords = 12224;          // 47.75 KiB of LDS: with the slices, two workgroups still fit a CU
constexpr int kHotBits = kHotWords * 32;  // 391168 hot vertices
constexpr int64_t kHotMinEdges = 1 << 22;  // graphs from this size get the filter by default
constexpr int kHotMinTiles = 4;            // sub-tiles per share for the LDS copy to pay off
constexpr int kLiteShares = 32;            // fewer active workgroups: no hot or frontier bit upkeep
constexpr int kHotTarget = -2;             // a gathered edge whose target is hot, id not yet looked up

// LDS words used by the level loop (the two layouts share one allocation).
constexpr int kLdsSmall = 3 * kSmallN + 1;             // group levels' frontier (v, rs, ex)
constexpr int kLdsLarge = 2 * 2 * kSlice + kHotWords;  // double-buffered sub-tile slices (ex, rs - ex), hot bits
constexpr int kLdsWords = (kLdsSmall > kLdsLarge ? kLdsSmall : kLdsLarge) + 2 * kWaves + 8;

// ---- device control block --------------------------------------------------------------
// Every field is accessed with agent-scope atomics (coherent across XCDs).
struct Ctrl {
    unsigned long long bar;   // grid-barrier arrivals, monotone within a launch
    // group levels, the frontier of level l in slot l % 3: (edges << 32) | entries,
    // (vertices reached << 32) | entries spilled past a member's LDS, the largest member's
    // edges, and the next free position of the global entry arrays
    unsigned long long g_ne[3];
    unsigned long long g_rs[3];
    unsigned long long g_mx[3];
    unsigned long long g_pos[3];
    unsigned int unused[2];
    int nl[2];                // next frontier size (vertices of degree >= 1), per parity
    int el[2];                // next frontier edge total, per parity
    int kept[2];              // vertices reaching that level (any degree), per parity
    int levels;               // frontiers processed (max level + 1)
    int error;                // 0, or a BFS_E* code set on the device
    int small_levels;         // levels run by the group of workgroups
    int resume;               // level at which the full grid resumes
    int heartbeat;            // bumped by the group so waiting workgroups keep waiting
    int plain_next;           // PLAIN mode: next-frontier counter
    int b_nact[2];            // batched: active vertices of a level, per parity
    int b_eact[2];            // batched: their edge total, per parity
    int blevel;               // batched: level whose expansion runs next
    int bdone;                // batched: no active vertex left (or overflow)
    int batch_overflow;       // batched: a level reached 255
    int r_nl, r_el, r_kept;   // frontier handed back by the group (level = resume)
    int nz_count;             // batched: vertices of degree >= 1
    int bu_levels;            // levels run bottom-up
    int pad[4];
};

// State of the grid barrier grouped by XCD (accelerator die).  Each counter
// sits on a line of its own, so the XCDs' arrivals and polls do not meet on
// one address.
constexpr int kMaxXcd = 16;   // XCC ids are four bits wide
constexpr int kXLine = 32;    // 64-bit words between two counters (256 bytes)
struct XBar {
    unsigned long long wgs[kMaxXcd * kXLine];     // workgroups of the launch on each XCD
    unsigned long long arrive[kMaxXcd * kXLine];  // arrivals on each XCD, monotone within a launch
    unsigned long long gen[kMaxXcd * kXLine];     // barriers completed, one copy per XCD
    unsigned long long top[kXLine];               // XCD groups complete, monotone within a launch
    unsigned long long pcnt[kXLine];              // arrivals at a barrier of a lite level's workgroups
    unsigned long long pgen[kMaxXcd * kXLine];    // generation of those barriers, one copy per XCD
};

// What the persistent level loop needs only now and then (per level, per barrier, per stretch of
// group levels): behind one pointer, filled by k_prep, so that the loop does not keep these
// values in scalar registers throughout.
struct Aux {
    int32_t* stat_nl;
    int32_t* stat_el;
    uint64_t* stat_ts;
    const int32_t* roots;
    XBar* xbar;
    uint32_t* snap;
    int32_t* gv[2];
    int32_t* grs[2];
    int32_t* gd[2];
    int32_t small_edges;
    int32_t bu_alpha;
    int32_t bu_beta;
    int32_t insensitive;
    int32_t group;
};

struct Params {
    // graph
    const int32_t* offsets;
    const int32_t* cols;
    const int32_t* colx;      // per edge: the target, or -1 - its hot number (null: no filter)
    const int32_t* hot_vid;   // vertex id of each hot number
    uint32_t* hot[2];         // visited bits of hot vertices: levels <= l in hot[l & 1]
    int32_t hot_words;        // words of each hot array (0: no filter)
    int32_t hot_count;        // hot numbers in use (entries of hot_vid)
    int32_t n;
    int64_t m;
    // outputs (caller-owned)
    int32_t* level;
    int32_t* parent;          // may be null
    // workspace
    uint32_t* bitmap;         // visited filter, 1 bit per vertex
    int32_t* owner;           // owning candidate slot per vertex
    int32_t* f_rs[2];         // frontier row starts, per parity
    int32_t* f_ex[2];         // frontier exclusive degree sums (+ total), per parity
    int32_t* f_v[2];          // frontier vertex ids, per parity (written only if non-null)
    int32_t* tstart[2];       // sub-tile start points, per parity
    int32_t* cand;            // private queues: share b owns cand[tb*kGrain, te*kGrain)
    int64_t cand_cap;         // entries of cand
    int32_t* cnt;             // queue length per share
    unsigned long long* desc[2];  // look-back descriptors per share, per parity
    Ctrl* ctrl;
    XBar* xbar;               // persistent loop's barrier state
    int32_t* stat_nl;
    int32_t* stat_el;
    uint64_t* stat_ts;        // per level: start, start of compaction, end (s_memrealtime ticks)
    // roots
    const int32_t* roots;     // device array, or null for a single root
    int32_t single_root;
    int32_t nroots;
    // group levels: next-frontier entries (vertex, row start, degree), kGroupCap per parity
    int32_t* gv[2];
    int32_t* grs[2];
    int32_t* gd[2];
    int32_t group;            // workgroups of the group (at most the grid)
    // tuning
    int32_t small_edges;      // 0 disables group levels
    int32_t push_edges;       // levels with at most this many edges push parents, larger ones pull
    // direction optimisation (persistent loop only)
    uint32_t* fbits[2];       // frontier bits: exactly the level-l vertices of degree >= 1 in fbits[l & 1]
    uint32_t* snap;           // visited bits at the start of a dense level
    int32_t direction;        // 1: levels may run bottom-up
    int32_t fb_pull;          // top-down persistent loop: keep frontier bits, pull parents against them
    int32_t insensitive;      // persistent loop: every level is split over every workgroup (P_l = P)
    int32_t dense_edges;      // top-down persistent loop: pull levels with at least this many edges keep
                              // the new frontier as bits (0: never)
    int32_t bu_alpha;         // go bottom-up when e_l * alpha > edges of unreached vertices
    int32_t bu_beta;          // return top-down when n_l * beta < n
    int32_t max_tiles;
    int32_t split_search;     // 1: each share finds its sub-tile start points by binary search
                              // instead of the compaction scattering them (Find-StartExpPoint)
    uint64_t spin_ticks;      // s_memrealtime ticks a wait may last without progress
    Aux* aux;                 // device copy of the fields above that the persistent loop reads
                              // through it (k_prep writes it)
};

// Batched multi-source search (up to 256 sources, 4 x 64-bit masks per vertex).
// The expansion's sub-tile (grain) and the dense update's tile are launch
// parameters chosen per workspace: grain = kBlock * bvt edges with bvt in
// {1, 2, 4}, update tile = kBlock * uv vertices with uv in {2, 4, 8}.
constexpr int kBVTMin = 1, kBVTMax = 4;
constexpr int kUVMin = 2, kUVMax = 8;
constexpr int kBVTDefault = 2;            // 1024 edges per sub-tile
constexpr int kUVDefault = 4;             // 2048 vertices per update tile
constexpr int kNzTile = 2048;             // vertices per tile of the one-off degree >= 1 listing

// Per-run arguments of a batched search, read by the kernels from device
// memory so that one captured level loop serves every run of a workspace.
struct BatchArgs {
    uint8_t* level;           // [n][k], 255 = unreached
    int32_t k;                // sources in this batch (1..256)
    int32_t words;            // mask words in use, ceil(k / 64)
    int32_t pull_edges;       // levels with more active edges pull instead of pushing
    int32_t pad;
};

struct BatchParams {
    const int32_t* offsets;
    const int32_t* cols;
    int32_t n;
    int64_t m;
    const BatchArgs* args;    // this run's output, k and thresholds
    unsigned long long* fr;   // frontier masks [n][4]
    unsigned long long* nx;   // next masks [n][4] (all zero between levels)
    unsigned long long* vis;  // visited masks [n][4]
    int32_t* act[2];          // active vertices, per level parity
    int32_t* act_rs[2];       // their row starts
    int32_t* act_ex[2];       // their exclusive degree sums (+ total)
    int32_t* act_ts[2];       // sub-tile start points over the active edges
    uint32_t* act_bits;       // active bitmap of the level being expanded
    int32_t* nz_v;            // vertices of degree >= 1, ascending (static per graph)
    int32_t* nz_ts;           // sub-tile start points over all edges [0, m) in nz_v
    unsigned long long* desc[2];  // look-back descriptors of the update tiles, per parity
    const int32_t* sources;   // the k sources (device)
    // hot-vertex numbering of the graph (null colx: none): pull levels read the neighbour stream
    // colx and gather a hot neighbour's frontier masks from the compact fr_hot[hot_count][4]
    const int32_t* colx;
    const int32_t* hot_vid;
    int32_t hot_count;
    unsigned long long* fr_hot;
    Ctrl* ctrl;
    int32_t* stat_nl;
    int32_t* stat_el;
    int32_t max_tiles;        // entries of act_ts / nz_ts (sized for the finest grain)
    int32_t utiles;           // update tiles, ceil(n / (kBlock * uv))
    int32_t desc_cap;         // entries of each descriptor array
    int32_t bvt;              // edges per thread in one expansion sub-tile
    int32_t uv;               // vertices per thread in one update tile
    uint64_t spin_ticks;
};

// ---- host-side launchers (bfs_kernels.hip) ---------------------------------------------
int persistent_grid_capacity(int device);   // workgroups that can be co-resident
hipError_t launch_prep(const Params& p, int prep_shares, bool fill_parent, hipStream_t s);
hipError_t launch_hot_gather(const int32_t* cols, int64_t m, const int32_t* hidx, int32_t* colx, int32_t n,
                             hipStream_t s);
hipError_t launch_persistent(const Params& p, int grid, hipStream_t s);
hipError_t launch_scrub(const Params& p, hipStream_t s);
hipError_t launch_status(const Ctrl* c, int32_t* out, hipStream_t s);
hipError_t launch_level_roots(const Params& p, int shares, hipStream_t s);
hipError_t launch_level_compact(const Params& p, int l, int ntiles, int shares, hipStream_t s);
hipError_t launch_level_expand(const Params& p, int l, int ntiles, int shares, hipStream_t s);
hipError_t launch_parent(const Params& p, hipStream_t s);
hipError_t launch_plain_init(const Params& p, int32_t* fv0, hipStream_t s);
hipError_t launch_plain_level(const Params& p, int l, const int32_t* fv, int nf, int32_t* fv_next,
                              hipStream_t s);
hipError_t launch_prim_compact(const int32_t* offsets, int32_t n, const int32_t* owner,
                               const int32_t* cand, const int32_t* cnt, int32_t ntiles, int32_t* out_v,
                               int32_t* out_rs, int32_t* out_ex, int32_t* out_tstart, int32_t tstart_cap,
                               int32_t* totals, unsigned long long* desc, Ctrl* ctrl, uint32_t* bitmap,
                               hipStream_t s);

hipError_t launch_batch_setup(const BatchParams& p, int grid, hipStream_t s);
hipError_t launch_batch_args(BatchArgs* dst, const BatchArgs& a, hipStream_t s);
hipError_t launch_batch_start(const BatchParams& p, hipStream_t s);
hipError_t launch_batch_level(const BatchParams& p, int grid, hipStream_t s);
hipError_t launch_batch_finish(const BatchParams& p, hipStream_t s);
int batch_grid_capacity(int device, int bvt);

// bfs_sort.hip: every row of the CSR sorted ascending into cols_out (synchronous on s)
hipError_t sort_rows_device(const int32_t* offsets, const int32_t* cols_in, int32_t* cols_out, int32_t n, int64_t m,
                            hipStream_t s);

}  // namespace s3bfs
