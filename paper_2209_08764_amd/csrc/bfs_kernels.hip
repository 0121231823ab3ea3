// HIP kernels of the S3BFS level loop for gfx950 (wave64, CDNA4).
//
// One level of the paper's Figure 1 maps onto two phases:
//
//   expand   Each share of kGrain consecutive frontier edges (a "tile",
//            the paper's per-thread share of e_l) is scanned by one
//            workgroup.  The tile's slice of the frontier's degree prefix
//            sums is staged in LDS; each wave finds the vertices owning its
//            rows of 64 edges there, every lane reads its neighbour word, filters
//            the target through the visited filters, and records each new
//            vertex (EXPLORE-VERTEX, with the benign race of the Algorithm
//            paragraph): owner = its candidate slot and a place in the
//            tile's private queue.
//   compact  Each tile's queue keeps the entries whose slot still owns the
//            vertex (Owner de-duplication), reads the survivors' degrees,
//            and a decoupled look-back scan over tiles gives every survivor
//            its position in the next frontier and its exclusive degree sum
//            (the Sizes prefix sum and linearisation fused with the next
//            level's degree gather and Parallel-Prefix-Sum).  Each survivor
//            then writes itself as the start point of every share that
//            begins inside its edge range (Find-StartExpPoint's scatter).
//
// Dense levels (most edges scanned) record new vertices by their visited
// bits alone and linearise them by vertex range instead of by queue.  The
// persistent kernel runs all levels in one launch with grid barriers between
// phases; only ceil(e_l / kGrain) workgroups have work in a phase
// (P_l = min(P, W_l)), levels with few workgroups synchronise only those, and
// while a level is small a group of workgroups runs it out of LDS with one
// barrier of its own per level, so the rest of the grid idles: a level
// occupies only as many cores as its work can use.
#include "bfs_device.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s3bfs {

// Marks every share that starts inside [e, e + d) as starting at frontier entry pos
// (Find-StartExpPoint).  With split_search the expansion finds the start points
// by binary search instead (search_starts), and nothing is scattered.
__device__ __forceinline__ void scatter_starts(const Params& p, int32_t* tstart, int pos, int e, int d) {
    if (p.split_search) return;
    int64_t t = ((int64_t)e + kGrain - 1) / kGrain;
    int64_t tend = ((int64_t)e + d + kGrain - 1) / kGrain;
    if (t < 0 || tend > p.max_tiles) {
        flag_internal(p.ctrl);
        return;
    }
    for (; t < tend; ++t) tstart[t] = pos;
}

struct Lds {
    int w[kLdsWords];
};

__device__ __forceinline__ int* lds_wave(int* lds) { return lds + kLdsWords - 2 * kWaves - 8; }
__device__ __forceinline__ int* lds_wave2(int* lds) { return lds + kLdsWords - kWaves - 8; }
__device__ __forceinline__ int* lds_misc(int* lds) { return lds + kLdsWords - 8; }

// Share b of P: the contiguous run of sub-tiles [tb, te) of the level's
// ntiles (the paper's (almost) equal division of e_l among P_l threads,
// rounded to whole sub-tiles; shares differ by at most one sub-tile).  Its
// private queue is cand[tb * kGrain, te * kGrain).
__device__ __forceinline__ void share_range(int b, int P, int ntiles, int* tb, int* te) {
    *tb = (int)(((int64_t)b * ntiles) / P);
    *te = (int)(((int64_t)(b + 1) * ntiles) / P);
}

// The alternative to the scatter: before its expansion, share b finds the
// start point of each of its sub-tiles [tb, te] (te too when another sub-tile
// follows) by a binary search of the level's exclusive degree sums: the last
// frontier entry j with f_ex[j] <= t * kGrain.  One search per lane, all of
// them in flight together.  Called by the whole workgroup.
__device__ __forceinline__ void search_starts(const Params& p, int l, int b, int P, int ntiles, int n_l) {
    int tb, te;
    share_range(b, P, ntiles, &tb, &te);
    const int tend = te < ntiles ? te : ntiles - 1;
    const int32_t* fex = p.f_ex[l & 1];
    int32_t* tst = p.tstart[l & 1];
    const int steps = n_l > 1 ? 32 - __builtin_clz((unsigned)(n_l - 1)) : 0;
    for (int t = tb + (int)threadIdx.x; t <= tend; t += kBlock) {
        const int64_t g = (int64_t)t * kGrain;
        int lo = 0, hi = n_l;  // f_ex[lo] <= g < f_ex[hi] (f_ex[n_l] = e_l)
        for (int k = 0; k < steps; ++k) {
            const int mid = (lo + hi) >> 1;
            const bool right = (int64_t)fex[mid] <= g;
            lo = right ? mid : lo;
            hi = right ? hi : mid;
        }
        tst[t] = lo;
    }
    __syncthreads();  // full: the expansion reads these entries from global memory
}

// Parent of a vertex v reached at level l + 1 is its smallest-id neighbour
// at level l.  Two equivalent ways to get it, chosen per level:
//  push  (levels with few edges) every scanned edge (u, v) whose target is
//        unsettled does an atomic minimum parent[v] = min(parent[v], u); all
//        level-l neighbours of v are scanned in this level, and the order of
//        the minima does not matter;
//  pull  (large levels, where new vertices have many level-l neighbours)
//        once level l + 1 is final, v's sorted row is read until the first
//        neighbour at level l: level[c] == l, or its bit in the frontier
//        bits of level l where the persistent loop keeps them exact.  A lane
//        tests kPullScan neighbours; longer rows go to the whole workgroup
//        (first_parent_wg).
__device__ __forceinline__ void parent_push(const Params& p, int v, int u) {
    __hip_atomic_fetch_min(reinterpret_cast<unsigned*>(p.parent) + v, (unsigned)u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool frontier_bit(const uint32_t* fb, int c) { return (fb[c >> 5] >> (c & 31)) & 1u; }

// Whether c is at level l: its frontier bit, or its level where the bits are not kept.
__device__ __forceinline__ bool at_level(const Params& p, int c, int l, const uint32_t* fb) {
    return fb ? frontier_bit(fb, c) : p.level[c] == l;
}

// First neighbour at level l among the first kPullScan of the row, -2 if
// none there but the row is longer, -1 if the row has none at all.
__device__ __forceinline__ int first_parent_lane(const Params& p, int rs, int d, int l, const uint32_t* fb) {
    const int end = rs + min(d, kPullScan);
    for (int e = rs; e < end; e += 4) {
        int c[4];
        bool hit[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = e + q < end ? p.cols[e + q] : -1;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            hit[q] = (unsigned)c[q] < (unsigned)p.n && (fb ? frontier_bit(fb, c[q]) : p.level[c[q]] == l);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (hit[q]) return c[q];
    }
    return d > kPullScan ? -2 : -1;
}

// The whole workgroup reads the rest of a long row from position kPullScan,
// kBlock neighbours per step, and returns the first neighbour c with hit(c)
// (-1 if none).  Uniform arguments; s_red holds kWaves + 1 ints.
template <typename Hit>
__device__ __forceinline__ int first_hit_wg(const Params& p, int rs, int d, Hit hit_of, int* s_red) {
    for (int base = kPullScan; base < d; base += kBlock) {
        const int e = rs + base + threadIdx.x;
        int c = -1;
        bool hit = false;
        if (base + threadIdx.x < d) {
            c = p.cols[e];
            hit = (unsigned)c < (unsigned)p.n && hit_of(c);
        }
        const uint64_t bb = ballot(hit);
        if (lane_id() == 0) s_red[wave_id()] = bb ? wave_id() * 64 + __builtin_ctzll(bb) : INT32_MAX;
        lds_barrier();
        int first = INT32_MAX;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) first = min(first, s_red[w]);
        if (first != INT32_MAX && threadIdx.x == first) s_red[kWaves] = c;
        lds_barrier();
        const int found = s_red[kWaves];
        lds_barrier();
        if (first != INT32_MAX) return found;
    }
    return -1;
}

__device__ __forceinline__ int first_parent_wg(const Params& p, int rs, int d, int l, const uint32_t* fb, int* s_red) {
    if (fb) return first_hit_wg(p, rs, d, [&](int c) { return frontier_bit(fb, c); }, s_red);
    return first_hit_wg(p, rs, d, [&](int c) { return p.level[c] == l; }, s_red);
}

// Owner of each of this lane's kVT sub-tile positions g0 + i * kBlock +
// threadIdx.x: the last of the nv staged entries whose exclusive degree sum
// ex[] is at most the position.  The sums ascend strictly (every staged
// vertex has an edge) and ex[0] <= g0.  A wave owns rows of 64 consecutive
// positions and resolves each row together instead of searching per lane:
// ballots over 64 sampled sums, then over the stretch between two samples,
// give the entry o covering the row's first position q0; each later entry
// that starts inside the row sends a flag to the lane of its first position
// (ds_permute, which hands unaddressed lanes zero), and a lane's owner is o
// plus the starts at or before it.  Whole waves must call it; the code is
// branch-free per row, so the rows' LDS round trips overlap.
template <bool SMALL>  // SMALL: nv <= 64, the samples are all the entries
__device__ __forceinline__ void owners_of_rows_n(const int* ex, int nv, int g0, int* own) {
    const int lane = lane_id();
    const int s = (nv + 63) >> 6;  // sampling stride, 1..33 for nv <= kSlice
    // Every read is issued from a clamped index and every lane's value is
    // compared; lanes past the entries are masked out of the ballots (bitwise
    // tests, so that no read sits behind a branch).  The rows go step by step
    // together, so that their reads are in flight at once.
    const int x1 = ex[min(lane * s, nv - 1)];
    const bool in1 = lane * s < nv;
    int q0[kVT], o[kVT], xs[kVT];
    bool ins[kVT];
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        q0[i] = g0 + i * kBlock + wave_id() * 64;
        o[i] = (max((int)__popcll(ballot(in1 & (x1 <= q0[i]))), 1) - 1) * s;
        xs[i] = x1;
        ins[i] = in1;
    }
    if (!SMALL) {
        int x2[kVT];
#pragma unroll
        for (int i = 0; i < kVT; ++i) x2[i] = ex[min(o[i] + lane, nv - 1)];
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            o[i] += max((int)__popcll(ballot((lane < s) & (o[i] + lane < nv) & (x2[i] <= q0[i]))), 1) - 1;
            xs[i] = ex[min(o[i] + 1 + lane, nv - 1)];
            ins[i] = o[i] + 1 + lane < nv;
        }
    }
    int r[kVT];
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        const int d = xs[i] - q0[i];  // > 0 for the entries after o
        const bool send = ins[i] & (d >= 1) & (d < 64);
        r[i] = __builtin_amdgcn_ds_permute((send ? d : 0) << 2, send ? d : 0);
    }
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        const bool hit = (lane > 0) & (r[i] == lane);
        own[i] = min(o[i] + mbcnt(ballot(hit)) + (int)hit, nv - 1);
    }
}

__device__ __forceinline__ void owners_of_rows(const int* ex, int nv, int g0, int* own) {
    if (nv <= 64) owners_of_rows_n<true>(ex, nv, g0, own);
    else owners_of_rows_n<false>(ex, nv, g0, own);
}

// Issues the neighbour reads of this lane's kVT edges among [g0, g1) of the
// current frontier, whose entries [j0, j0 + nv) are staged in `sl` (ex | rs - ex):
// raw words of the neighbour stream into x (decode_tile interprets them) and
// bit i of *ok set where edge i exists; with `fv` also the frontier vertex
// each edge comes from (for pushed parents).  Every neighbour read is
// issued, from a clamped address where a lane has no edge, and nothing
// reads its result here: the reads stay in flight while the previous
// sub-tile is filtered, and the waits before that filtering can count them.
__device__ __forceinline__ void gather_tile(const Params& p, const int* sl, int nv, int g0, int g1, int* x,
                                            uint32_t* ok, const int32_t* fv, int j0, int* u) {
    int gg[kVT], own[kVT];
#pragma unroll
    for (int i = 0; i < kVT; ++i) gg[i] = min(g0 + i * kBlock + (int)threadIdx.x, g1 - 1);
    owners_of_rows(sl, nv, g0, own);
    const int32_t* src = p.colx ? p.colx : p.cols;
    // frontier vertices first (push levels only), then the neighbour words, which every
    // lane issues: a wait for anything issued before them can leave them in flight
    if (fv) {
#pragma unroll
        for (int i = 0; i < kVT; ++i) u[i] = fv[j0 + own[i]];
    }
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        const int g = g0 + i * kBlock + threadIdx.x;
        const int lo = own[i];
        const int idx = sl[kSlice + lo] + gg[i];
        const bool in = (unsigned)idx < (unsigned)p.m;
        if (g < g1 && in) m |= 1u << i;
        if (g < g1 && !in) flag_internal(p.ctrl);
        x[i] = __builtin_nontemporal_load(src + (in ? idx : 0));
    }
    *ok = m;
}

// Interprets the words gather_tile read: v = the target (-1: no edge, or a
// target outside [0, n)); with the hot-vertex filter a hot target comes
// back as kHotTarget with its hot number in h (-1 for the others), and
// expand_share resolves its id once the hot bits leave it open.
__device__ __forceinline__ void decode_tile(const Params& p, const int* x, uint32_t ok, int* v, int* h) {
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        v[i] = -1;
        h[i] = -1;
        if ((ok >> i) & 1u) {
            if (x[i] >= 0) {
                v[i] = x[i] < p.n ? x[i] : -1;
            } else if (p.colx && -1 - x[i] < p.hot_count) {
                h[i] = -1 - x[i];
                v[i] = kHotTarget;
            }
        }
    }
}

// ---- EXPLORE-VERTEX over one share ---------------------------------------------------------
// The share's sub-tiles are scanned in order, software-pipelined: while the
// neighbours of sub-tile t are filtered, the neighbour reads of sub-tile
// t + 1 are in flight and the frontier entries of sub-tile t + 2 are being
// fetched into registers.  Sub-tile t needs the frontier entries
// [tstart[t], tstart[t+1]] (at most kSlice of them, since every frontier
// vertex has an edge), staged in one of two LDS buffers; each wave maps its
// rows of 64 edges to entries there (owners_of_rows).  A target passes the visited
// filters (hot bits, then the visited bitmap) only if it was not reached
// before this level; push levels then test its level, since every edge into
// a vertex reached in this level offers its source.  A new vertex gets its
// visited bit and, except on dense levels (which record new vertices by
// their visited bits alone), owner = its queue slot and a place in the queue
// (the benign race: several lanes may append the same vertex).
//
// Hot-vertex filter: when the graph numbers its highest-degree vertices,
// each share with enough edges copies the visited bits of those vertices
// for levels <= l (hot[l & 1], untouched during level l) into LDS and tests
// hot targets there before anything else; new hot vertices go to
// hot[(l + 1) & 1], which the shares also merge hot[l & 1] into (not on lite
// levels, which leave the hot bits inexact).  A set bit still means the
// vertex was visited before this level, so results are unchanged.
__device__ void expand_share(const Params& p, int l, int b, int P, int ntiles, int n_l, int e_l, int* lds,
                             bool dense = false, bool lite = false) {
    int* s_wave = lds_wave(lds);
    uint32_t* hnext = nullptr;
    const uint32_t* hcur = nullptr;
    if (p.hot_words > 0) {
        hcur = p.hot[l & 1];
        hnext = p.hot[(l + 1) & 1];
        // a lite level (few workgroups) leaves the hot bits alone: they are then inexact
        const int w0 = (int)(((int64_t)b * p.hot_words) / P);
        const int w1 = lite ? w0 : (int)(((int64_t)(b + 1) * p.hot_words) / P);
        for (int w = w0 + threadIdx.x; w < w1; w += kBlock) {
            const uint32_t x = hcur[w];
            if (x) __hip_atomic_fetch_or(&hnext[w], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    int tb, te;
    share_range(b, P, ntiles, &tb, &te);
    if (tb >= te) {
        if (threadIdx.x == 0) p.cnt[b] = 0;
        return;
    }
    const bool use_hot = hcur && te - tb >= kHotMinTiles;  // LDS copy of the hot bits, else read in place
    uint32_t* s_hot = reinterpret_cast<uint32_t*>(lds + 4 * kSlice);
    const int par = l & 1;
    const int32_t* tst = p.tstart[par];
    const int32_t* fex = p.f_ex[par];
    const int32_t* frs = p.f_rs[par];
    const int32_t* fvp = (p.parent && e_l <= p.push_edges) ? p.f_v[par] : nullptr;  // push level
    const int qbase = tb * kGrain;
    int qn = 0;
    auto slice_end = [&](int t) { return t + 1 < ntiles ? tst[t + 1] : n_l - 1; };
    auto slice_ok = [&](int a, int z) { return a >= 0 && z < n_l && z >= a && z - a + 1 <= kSlice; };
    auto stage_slice = [&](int* buf, int a, int z) {
        for (int i = threadIdx.x; i <= z - a; i += kBlock) {
            const int e = fex[a + i];
            buf[i] = e;
            buf[kSlice + i] = frs[a + i] - e;
        }
    };
    int* buf0 = lds;
    int* buf1 = lds + 2 * kSlice;
    // prologue: slices of sub-tiles tb and tb + 1 in LDS, neighbours of tb in flight
    const int a0 = tst[tb], z0 = slice_end(tb);
    int a1 = z0, z1 = (tb + 1 < te) ? slice_end(tb + 1) : z0;
    bool bad = !slice_ok(a0, z0) || (tb + 1 < te && !slice_ok(a1, z1));
    if (!bad) {
        stage_slice(buf0, a0, z0);
        if (tb + 1 < te) stage_slice(buf1, a1, z1);
    }
    if (use_hot)
        for (int w = threadIdx.x; w < p.hot_words; w += kBlock) s_hot[w] = hcur[w];
    lds_barrier();
    // raw neighbour words of the sub-tile to filter next, which of them are edges, and
    // (push levels) their frontier entries' vertices
    int xc[kVT], uc[kVT];
    uint32_t okc = 0u;
#pragma unroll
    for (int i = 0; i < kVT; ++i) xc[i] = uc[i] = -1;
    if (!bad) gather_tile(p, buf0, z0 - a0 + 1, tb * kGrain, min(tb * kGrain + kGrain, e_l), xc, &okc, fvp, a0, uc);
    for (int t = tb; t < te && !bad; ++t) {
        int* cur1 = ((t + 1 - tb) & 1) ? buf1 : buf0;   // slice of sub-tile t + 1
        int* free2 = ((t - tb) & 1) ? buf1 : buf0;      // receives the slice of sub-tile t + 2
        // Sub-tile t's neighbour words (read during the previous sub-tile) are decoded
        // first.  Then the slice reads for sub-tile t + 2 go out, then the probes of
        // sub-tile t, then the neighbour reads for sub-tile t + 1, which every lane
        // issues: reads return in issue order, so waiting for the probes does not wait
        // for the neighbour reads behind them, and the slice reads ahead of the probes
        // may be skipped by lanes with no entry.  Hot targets are tested against the LDS
        // copy; one that passes is new to this level unless another edge found it
        // first, which its bit in hnext tells (pull levels); its id comes from hot_vid.
        // The other targets are tested against the visited bitmap.
        int vc[kVT], hc[kVT];
        decode_tile(p, xc, okc, vc, hc);
        // fetch the slice of sub-tile t + 2 into registers
        const bool has2 = t + 2 < te;
        const int a2 = z1, z2 = has2 ? slice_end(t + 2) : z1;
        const bool ok2 = !has2 || slice_ok(a2, z2);
        int pe[kPre], pr[kPre];
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
            const int i = threadIdx.x + r * kBlock;
            if (has2 && ok2 && i <= z2 - a2) {
                pe[r] = fex[a2 + i];
                pr[r] = frs[a2 + i];
            }
        }
        uint32_t pw[kVT];
        int hid[kVT];
        bool any_open = false;
#pragma unroll
        for (int i = 0; i < kVT; ++i) hid[i] = -1;
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            bool hot_open = false;
            if (hc[i] >= 0) {
                const uint32_t w = use_hot ? s_hot[hc[i] >> 5] : hcur[hc[i] >> 5];
                hot_open = !((w >> (hc[i] & 31)) & 1u);
                if (!hot_open) {
                    vc[i] = -1;
                    hc[i] = -1;
                }
            }
            any_open |= hot_open;
            const uint32_t* pa = (hot_open && !fvp) ? hnext + (hc[i] >> 5) : p.bitmap + (max(vc[i], 0) >> 5);
            pw[i] = *pa;
        }
        // ids of open hot targets, only in waves that have one (the reads behind stay
        // unconditional); a dense level needs none: its hot discoveries reach the visited
        // bitmap from the hot bits after the level (merge_hot_discoveries)
        if (!dense && ballot(any_open)) {
#pragma unroll
            for (int i = 0; i < kVT; ++i) hid[i] = p.hot_vid[hc[i] >= 0 ? hc[i] : 0];
        }
        // issue the neighbour reads of sub-tile t + 1
        int xn[kVT], un[kVT];
        uint32_t okn = 0u;
#pragma unroll
        for (int i = 0; i < kVT; ++i) xn[i] = un[i] = -1;
        if (t + 1 < te)
            gather_tile(p, cur1, z1 - a1 + 1, (t + 1) * kGrain, min((t + 1) * kGrain + kGrain, e_l), xn, &okn, fvp,
                        a1, un);
        // decide sub-tile t
        bool fresh[kVT];
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            const bool hot = hc[i] >= 0;
            if (hot) vc[i] = dense ? 0 : hid[i];  // dense: a stand-in id, used by nothing below
            // a push level tests an open hot target by its level below, like any other
            const bool seen = hot ? !fvp && ((pw[i] >> (hc[i] & 31)) & 1u) : ((pw[i] >> (vc[i] & 31)) & 1u);
            if (vc[i] >= 0 && seen) vc[i] = -1;
        }
        if (fvp) {
            // push level: every edge into an unsettled vertex offers its source as parent
#pragma unroll
            for (int i = 0; i < kVT; ++i) {
                fresh[i] = false;
                if (vc[i] >= 0) {
                    const int lv = p.level[vc[i]];
                    if (lv == -1) fresh[i] = true;
                    else if (lv != l + 1) vc[i] = -1;
                }
            }
#pragma unroll
            for (int i = 0; i < kVT; ++i)
                if (vc[i] >= 0) parent_push(p, vc[i], uc[i]);
        } else {
            // pull level: the bitmap holds every vertex visited before level l, so a
            // target that passed it is new; its level is written at de-duplication
            // (a target reached twice in this level is a duplicate the owner test drops)
#pragma unroll
            for (int i = 0; i < kVT; ++i) fresh[i] = vc[i] >= 0;
        }
        // A pull level sets the visited bit at discovery, so later edges into
        // the vertex stop at the bitmap; a push level must let every such edge
        // offer its source, so its bits are set at de-duplication instead.
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            if (fresh[i]) {
                if (fvp) p.level[vc[i]] = l + 1;
                else if (!dense || hc[i] < 0)
                    __hip_atomic_fetch_or(&p.bitmap[vc[i] >> 5], 1u << (vc[i] & 31), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                if (hnext && hc[i] >= 0 && !lite)
                    __hip_atomic_fetch_or(&hnext[hc[i] >> 5], 1u << (hc[i] & 31), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (!dense) {
            int slot[kVT];
            int wt = 0;
#pragma unroll
            for (int i = 0; i < kVT; ++i) {
                const uint64_t bb = ballot(fresh[i]);
                slot[i] = wt + mbcnt(bb);
                wt += __popcll(bb);
            }
            if (lane_id() == 0) s_wave[wave_id()] = wt;
            lds_barrier();
            int wbase = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const int x = s_wave[w];
                wbase += (w < wave_id()) ? x : 0;
                tot += x;
            }
#pragma unroll
            for (int i = 0; i < kVT; ++i) {
                if (fresh[i]) {
                    const int s = qbase + qn + wbase + slot[i];
                    p.owner[vc[i]] = s;
                    p.cand[s] = vc[i];
                }
            }
            qn += tot;
        }
        // publish the slice of sub-tile t + 2 (the buffer of sub-tile t is free)
        if (has2) {
            if (!ok2) {
                bad = true;
            } else {
#pragma unroll
                for (int r = 0; r < kPre; ++r) {
                    const int i = threadIdx.x + r * kBlock;
                    if (i <= z2 - a2) {
                        free2[i] = pe[r];
                        free2[kSlice + i] = pr[r] - pe[r];
                    }
                }
            }
        }
        a1 = a2;
        z1 = z2;
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            xc[i] = xn[i];
            uc[i] = un[i];
        }
        okc = okn;
        lds_barrier();
    }
    if (threadIdx.x == 0) {
        if (bad) flag_internal(p.ctrl);
        p.cnt[b] = qn;
    }
    lds_barrier();
}

// Pulls the parents of one chunk's new vertices (kVT per thread, v = -1 for
// none).  The first kFirst neighbours of every row are tested at once; the
// rows still open then go to a list in LDS, one per lane, so that no lane
// scans its rows one after another while the rest of its wave waits; a lane
// tests kPullScan more neighbours, and the few rows longer than that are
// scanned by one wave each, 64 neighbours per step.  Uses the LDS slice
// buffers; called by the whole workgroup.
__device__ __forceinline__ void pull_parents_chunk(const Params& p, const int* v, const int* rs, const int* d, int l,
                                                   const uint32_t* fpull, int* lds) {
    int* s_row = lds;                 // (v, row start, length) of the open rows, then of the long ones
    int* s_cnt = lds + 3 * kGrain;    // open rows, long rows
    if (threadIdx.x == 0) {
        s_cnt[0] = 0;
        s_cnt[1] = 0;
    }
    lds_barrier();
    constexpr int kFirst = 2;
    int c[kVT][kFirst];
    bool h[kVT][kFirst];
#pragma unroll
    for (int i = 0; i < kVT; ++i)
#pragma unroll
        for (int q = 0; q < kFirst; ++q) {
            // every lane reads, from a clamped position of its row (of row 0 for no row), and
            // masks afterwards, so that no read sits behind a branch
            const int x = p.cols[rs[i] + max(min(q, d[i] - 1), 0)];
            c[i][q] = ((v[i] >= 0) & (q < d[i])) ? x : -1;
        }
    if (fpull) {
#pragma unroll
        for (int i = 0; i < kVT; ++i)
#pragma unroll
            for (int q = 0; q < kFirst; ++q) {
                const int x = (unsigned)c[i][q] < (unsigned)p.n ? c[i][q] : 0;
                h[i][q] = (c[i][q] >= 0) & frontier_bit(fpull, x);
            }
    } else {
#pragma unroll
        for (int i = 0; i < kVT; ++i)
#pragma unroll
            for (int q = 0; q < kFirst; ++q) {
                const int x = (unsigned)c[i][q] < (unsigned)p.n ? c[i][q] : 0;
                h[i][q] = (c[i][q] >= 0) & (p.level[x] == l);
            }
    }
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        if (v[i] >= 0) {
            int f = -1;
#pragma unroll
            for (int q = kFirst - 1; q >= 0; --q)
                if (h[i][q]) f = c[i][q];
            if (f < 0 && d[i] > kFirst) {  // open: the rest of the row from position kFirst
                const int o = atomicAdd(&s_cnt[0], 1);
                s_row[3 * o] = v[i];
                s_row[3 * o + 1] = rs[i] + kFirst;
                s_row[3 * o + 2] = d[i] - kFirst;
            } else {
                p.parent[v[i]] = f;
            }
        }
    }
    lds_barrier();
    const int nopen = s_cnt[0];
    for (int j0 = 0; j0 < nopen; j0 += kBlock) {
        const int j = j0 + (int)threadIdx.x;
        int rv = -1, rr = 0, rd = 0;
        if (j < nopen) {
            rv = s_row[3 * j];
            rr = s_row[3 * j + 1];
            rd = s_row[3 * j + 2];
        }
        // this round's entries are all read before long rows are written over the list's
        // front (long-row slot < rows taken so far <= j0 + kBlock)
        lds_barrier();
        if (rv >= 0) {
            const int f = first_parent_lane(p, rr, rd, l, fpull);
            if (f == -2) {
                const int o = atomicAdd(&s_cnt[1], 1);
                s_row[3 * o] = rv;
                s_row[3 * o + 1] = rr;
                s_row[3 * o + 2] = rd;
            } else {
                p.parent[rv] = f;
            }
        }
    }
    lds_barrier();
    const int nlong = s_cnt[1];
    for (int o = wave_id(); o < nlong; o += kWaves) {
        const int hv = s_row[3 * o], hrs = s_row[3 * o + 1], hd = s_row[3 * o + 2];
        int f = -1;
        for (int base = kPullScan; base < hd; base += 64) {
            const int q = base + lane_id();
            int x = -1;
            bool hit = false;
            if (q < hd) {
                x = p.cols[hrs + q];
                hit = (unsigned)x < (unsigned)p.n && at_level(p, x, l, fpull);
            }
            const uint64_t bb = ballot(hit);
            if (bb) {
                f = __shfl(x, __builtin_ctzll(bb));
                break;
            }
        }
        if (lane_id() == 0) p.parent[hv] = f;
    }
    lds_barrier();
}

// ---- de-duplication and linearisation of one share's queue -----------------------------------
// Pass 1 keeps queue entries whose slot still owns the vertex (Owner[v] = i).
// On pull levels the expansion left levels unwritten, so pass 1 also drops
// vertices already reached and writes level l + 1 for the others; on push
// levels and for the roots it sets their visited bits instead.  It compacts
// the survivors of degree >= 1 in place; the share's (count, edge total) then gets its exclusive prefix by
// decoupled look-back over the shares (the Sizes prefix sum).  Pass 2 writes
// the survivors to the next frontier with their exclusive degree sums and
// the start points of the next level's sub-tiles.  l = -1 compacts the roots.
__device__ bool compact_share(const Params& p, int l, int b, int P, int ntiles, bool pull_parents, bool set_bits,
                              int* lds, bool after_bottom_up = false, const uint32_t* fpull = nullptr,
                              bool keep_fb = true) {
    int* s_wave = lds_wave(lds);
    int* s_wave2 = lds_wave2(lds);
    int* s_b = lds_misc(lds);
    const int par = l & 1;
    const int np = (l + 1) & 1;
    // levels already written at expansion (push levels, roots, bottom-up levels); a
    // bottom-up level has no duplicates and has set the visited and frontier bits
    const bool settle = set_bits || l < 0 || after_bottom_up;
    const bool dedup = !after_bottom_up;
    int tb, te;
    share_range(b, P, ntiles, &tb, &te);
    const int qbase = tb * kGrain;
    int qn = tb < te ? p.cnt[b] : 0;
    if (qn < 0 || qn > (te - tb) * kGrain) {
        if (threadIdx.x == 0) flag_internal(p.ctrl);
        qn = 0;
    }
    // pass 1; a queue of one chunk keeps its survivors in registers for pass 2
    const bool one = qn <= kGrain;
    int kv[kVT], krs[kVT], kd[kVT], kpos0 = 0, ke0 = 0;
#pragma unroll
    for (int i = 0; i < kVT; ++i) {  // an empty queue (qn = 0) runs no chunk: no entries then
        kv[i] = -1;
        krs[i] = 0;
        kd[i] = 0;
    }
    int surv = 0, degsum = 0, raw = 0;
    for (int c0 = 0; c0 < qn; c0 += kGrain) {
        int v[kVT], d[kVT], rs[kVT];
        int tc = 0, ts = 0, tr = 0;
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            const int idx = c0 + threadIdx.x * kVT + i;
            v[i] = -1;
            if (idx < qn) {
                const int vv = p.cand[qbase + idx];
                if ((unsigned)vv >= (unsigned)p.n) flag_internal(p.ctrl);
                else if (!dedup || (p.owner[vv] == qbase + idx && (settle || p.level[vv] == -1))) v[i] = vv;
            }
        }
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            d[i] = 0;
            rs[i] = 0;
            if (v[i] >= 0) {
                if (!settle) p.level[v[i]] = l + 1;
                rs[i] = p.offsets[v[i]];
                d[i] = p.offsets[v[i] + 1] - rs[i];
                ++tr;
                if (set_bits)  // roots and push levels; pull levels set bits at discovery
                    __hip_atomic_fetch_or(&p.bitmap[v[i] >> 5], 1u << (v[i] & 31), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                // frontier bits of level l + 1, for a bottom-up step or the next level's pulls
                if ((p.direction || (p.fb_pull && keep_fb)) && d[i] > 0 && !after_bottom_up)
                    __hip_atomic_fetch_or(&p.fbits[np][v[i] >> 5], 1u << (v[i] & 31), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                if (d[i] > 0) { ++tc; ts += d[i]; }
            }
        }
        int C, S, R;
        const int pos0 = block_excl_scan(tc, s_wave, &C);
        const int e0 = block_excl_scan(ts, s_wave2, &S);
        block_excl_scan(tr, s_wave, &R);
        if (one) {
#pragma unroll
            for (int i = 0; i < kVT; ++i) {
                // a slot without an entry has row start and degree 0, as the parent pull's
                // clamped reads require
                kv[i] = v[i] >= 0 && d[i] > 0 ? v[i] : -1;
                krs[i] = kv[i] >= 0 ? rs[i] : 0;
                kd[i] = kv[i] >= 0 ? d[i] : 0;
            }
            kpos0 = pos0;
            ke0 = e0;
        } else {
            // in place: every read of this chunk fed the scans, so it completed before their barriers
            int pos = surv + pos0;
#pragma unroll
            for (int i = 0; i < kVT; ++i)
                if (v[i] >= 0 && d[i] > 0) p.cand[qbase + pos++] = v[i];
        }
        surv += C;
        degsum += S;
        raw += R;
        lds_barrier();  // the next chunk's queue entries lie beyond every position written here
    }
    // Sizes prefix sum over the shares
    if (wave_id() == 0) {
        int pc = 0, ps = 0;
        const bool okw = lookback_wave(p.desc[par], b, surv, degsum, p.ctrl, p.spin_ticks, &pc, &ps);
        if (threadIdx.x == 0) {
            s_b[0] = pc;
            s_b[1] = ps;
            s_b[2] = okw;
            if (raw) __hip_atomic_fetch_add(&p.ctrl->kept[np], raw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (okw && b == P - 1) {
                st_rel(&p.ctrl->nl[np], pc + surv);
                st_rel(&p.ctrl->el[np], ps + degsum);
                if (pc + surv <= p.n) p.f_ex[np][pc + surv] = ps + degsum;
                else flag_internal(p.ctrl);
            }
        }
    }
    __syncthreads();  // full: pass 2 reads queue entries other lanes compacted in pass 1
    const int pc = s_b[0], ps = s_b[1];
    const bool ok = s_b[2] != 0;
    lds_barrier();
    if (!ok) return false;
    // pass 2
    const bool pull = p.parent && l >= 0 && pull_parents;
    if (one) {
        // the survivors are this thread's own from pass 1, in the order pass 1 counted them
        int pos = pc + kpos0, e = ps + ke0;
        if (pull && surv > 0) pull_parents_chunk(p, kv, krs, kd, l, fpull, lds);  // surv: uniform
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            if (kv[i] >= 0) {
                if ((unsigned)pos < (unsigned)p.n) {
                    p.f_v[np][pos] = kv[i];
                    p.f_rs[np][pos] = krs[i];
                    p.f_ex[np][pos] = e;
                    scatter_starts(p, p.tstart[np], pos, e, kd[i]);
                } else {
                    flag_internal(p.ctrl);
                }
                e += kd[i];
                ++pos;
            }
        }
        return true;
    }
    int run_e = 0;
    for (int c0 = 0; c0 < surv; c0 += kGrain) {
        int v[kVT], rs[kVT], d[kVT];
        int ts = 0;
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            const int idx = c0 + threadIdx.x * kVT + i;
            v[i] = -1;
            d[i] = 0;
            rs[i] = 0;
            if (idx < surv) {
                v[i] = p.cand[qbase + idx];
                rs[i] = p.offsets[v[i]];
                d[i] = p.offsets[v[i] + 1] - rs[i];
                ts += d[i];
            }
        }
        int S;
        int e = ps + run_e + block_excl_scan(ts, s_wave, &S);
        int pos = pc + c0 + threadIdx.x * kVT;
        if (pull) pull_parents_chunk(p, v, rs, d, l, fpull, lds);
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            if (v[i] >= 0) {
                if ((unsigned)pos < (unsigned)p.n) {
                    p.f_v[np][pos] = v[i];
                    p.f_rs[np][pos] = rs[i];
                    p.f_ex[np][pos] = e;
                    scatter_starts(p, p.tstart[np], pos, e, d[i]);
                } else {
                    flag_internal(p.ctrl);
                }
                e += d[i];
            }
            ++pos;
        }
        run_e += S;
    }
    return true;
}

// Compaction of a dense level.  There the expansion only sets each new
// vertex's visited bit instead of appending it to a private queue, and the
// level's new vertices are the bits set since the snapshot taken at its
// start: duplicates merge in the bitmap and the frontier comes out in vertex
// order, so the next level reads its rows, and this level pulls its parents,
// in the order they lie in memory.  Share b of P takes a range of whole
// kGrain-vertex chunks.  Pass 1 writes level l + 1 of every new vertex, the
// new-vertex words into fbits[(l + 1) & 1] (the next level's exact frontier
// bits), and counts the share's frontier entries (degree >= 1) and their
// edges; the look-back over the shares gives their offsets (the Sizes prefix
// sum); pass 2 writes the entries, the start points of the next level's
// sub-tiles and the pulled parents.
// Inputs of one dense-compaction chunk for this thread's kVT consecutive
// vertices from v: the word of their new-vertex bits (visited now and not at
// the level's start) and kVT + 1 row offsets.  Read by
// every lane from clamped addresses, so a chunk can be fetched while the
// previous one is processed and the wait for it counts exactly.
struct DenseIn {
    uint32_t w;
    int off[kVT + 1];
};
__device__ __forceinline__ DenseIn dense_load(const Params& p, int v) {
    DenseIn r;
    const int vb = min(v, p.n - 1);  // n >= 1; a vertex below n keeps its own data
    r.w = p.bitmap[vb >> 5] & ~p.aux->snap[vb >> 5];
#pragma unroll
    for (int k = 0; k <= kVT; ++k) r.off[k] = p.offsets[min(vb + k, p.n)];
    return r;
}

__device__ bool dense_compact_share(const Params& p, int l, int b, int P, int* lds, const uint32_t* fpull) {
    int* s_wave = lds_wave(lds);
    int* s_wave2 = lds_wave2(lds);
    int* s_b = lds_misc(lds);
    const int par = l & 1;
    const int np = (l + 1) & 1;
    uint32_t* fb = p.fbits[np];
    const int64_t chunks = ((int64_t)p.n + kGrain - 1) / kGrain;
    const int v0 = (int)(chunks * b / P * kGrain);
    const int v1 = (int)min((int64_t)p.n, chunks * (b + 1) / P * kGrain);
    // pass 1: thread t takes the kVT consecutive vertices from base + t * kVT; the next
    // chunk's bits and offsets are in flight while this one is counted
    const int tv = (int)threadIdx.x * kVT;
    int tc = 0, ts = 0, tr = 0;
    DenseIn cur = dense_load(p, v0 + tv);
    for (int base = v0; base < v1; base += kGrain) {
        const DenseIn nxt = dense_load(p, base + kGrain + tv);
        if (((base + tv) & 31) == 0 && base + tv < v1) fb[(base + tv) >> 5] = cur.w;  // one lane per word
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            const int v = base + tv + i;
            if (v < v1 && ((cur.w >> (v & 31)) & 1u)) {
                p.level[v] = l + 1;
                const int d = cur.off[i + 1] - cur.off[i];
                ++tr;
                if (d > 0) { ++tc; ts += d; }
            }
        }
        cur = nxt;
    }
    int surv, degsum, raw;
    block_excl_scan(tc, s_wave, &surv);
    block_excl_scan(ts, s_wave2, &degsum);
    block_excl_scan(tr, s_wave, &raw);
    if (wave_id() == 0) {
        int pc = 0, ps = 0;
        const bool okw = lookback_wave(p.desc[par], b, surv, degsum, p.ctrl, p.spin_ticks, &pc, &ps);
        if (threadIdx.x == 0) {
            s_b[0] = pc;
            s_b[1] = ps;
            s_b[2] = okw;
            if (raw) __hip_atomic_fetch_add(&p.ctrl->kept[np], raw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (okw && b == P - 1) {
                st_rel(&p.ctrl->nl[np], pc + surv);
                st_rel(&p.ctrl->el[np], ps + degsum);
                if (pc + surv <= p.n) p.f_ex[np][pc + surv] = ps + degsum;
                else flag_internal(p.ctrl);
            }
        }
    }
    __syncthreads();
    const int pc = s_b[0], ps = s_b[1];
    const bool ok = s_b[2] != 0;
    lds_barrier();
    if (!ok) return false;
    // pass 2: the same vertices in the same order
    const bool pull = p.parent != nullptr;
    int run_c = 0, run_e = 0;
    cur = dense_load(p, v0 + tv);
    for (int base = v0; base < v1; base += kGrain) {
        const DenseIn nxt = dense_load(p, base + kGrain + tv);
        int v[kVT], rs[kVT], d[kVT];
        int cc = 0, cs = 0;
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            const int vv = base + tv + i;
            v[i] = -1;
            rs[i] = d[i] = 0;
            const int dd = cur.off[i + 1] - cur.off[i];
            if (vv < v1 && ((cur.w >> (vv & 31)) & 1u) && dd > 0) {
                v[i] = vv;
                rs[i] = cur.off[i];
                d[i] = dd;
                ++cc;
                cs += dd;
            }
        }
        int C, S;
        int pos = pc + run_c + block_excl_scan(cc, s_wave, &C);
        int e = ps + run_e + block_excl_scan(cs, s_wave2, &S);
        if (pull) pull_parents_chunk(p, v, rs, d, l, fpull, lds);
#pragma unroll
        for (int i = 0; i < kVT; ++i) {
            if (v[i] >= 0) {
                if ((unsigned)pos < (unsigned)p.n) {
                    p.f_v[np][pos] = v[i];
                    p.f_rs[np][pos] = rs[i];
                    p.f_ex[np][pos] = e;
                    scatter_starts(p, p.tstart[np], pos, e, d[i]);
                } else {
                    flag_internal(p.ctrl);
                }
                e += d[i];
                ++pos;
            }
        }
        run_c += C;
        run_e += S;
        cur = nxt;
    }
    return true;
}

// Shares of a dense level's compaction: whole kGrain-vertex chunks, at most
// one share per workgroup and per descriptor.
__device__ __forceinline__ int dense_shares(const Params& p, int G) {
    const int64_t chunks = ((int64_t)p.n + kGrain - 1) / kGrain;
    return (int)min(min((int64_t)G, (int64_t)p.max_tiles), max(chunks, (int64_t)1));
}

// ---- bottom-up step (direction optimisation) ----------------------------------------------
// Instead of scanning the frontier's edges, every unreached vertex of this
// share's vertex range [tb * kGrain, te * kGrain) scans its sorted row for the
// first neighbour in the frontier (fbits[l & 1]); if there is one it is at
// level l + 1 and that neighbour is its smallest-id parent.  Each vertex is
// handled by one lane, so there are no duplicates.  Found vertices get their
// visited and frontier bits at once and go to the share's queue, whose length
// and edge total the share leaves in cnt[b] and cnt[max_tiles + b]; the queue
// is linearised only if the next level runs top-down.  A lane tests
// kPullScan neighbours; longer rows go to the whole workgroup.
// Vertex v reached from u at level l + 1 (where ok): level, parent, visited
// and frontier bits, and a slot of the share's queue; the wave reserves its
// slots with one LDS atomic.  With `packed` the wave's 64 vertices are
// consecutive from a multiple of 32, so each half-wave's bits form one word
// and go out as one atomic instead of 32 on the same address.
__device__ __forceinline__ void bu_settle(const Params& p, int l, int qbase, int* s_cnt, int v, int u, bool ok,
                                          bool packed) {
    const uint64_t bb = ballot(ok);
    int wbase = 0;
    if (lane_id() == 0 && bb) wbase = atomicAdd(s_cnt, __popcll(bb));
    wbase = __shfl(wbase, 0);
    uint32_t* fbn = p.fbits[(l + 1) & 1];
    if (ok) {
        const int slot = qbase + wbase + mbcnt(bb);
        p.level[v] = l + 1;
        if (p.parent) p.parent[v] = u;
        p.cand[slot] = v;
        if (!packed) {
            __hip_atomic_fetch_or(&p.bitmap[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_or(&fbn[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (packed && (lane_id() & 31) == 0) {
        const uint32_t word = (uint32_t)(bb >> (lane_id() & 32));
        if (word) {
            __hip_atomic_fetch_or(&p.bitmap[v >> 5], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_or(&fbn[v >> 5], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__device__ __forceinline__ void bottom_up_share(const Params& p, int l, int b, int P, int ntiles, int* lds) {
    constexpr int kBU = 4;  // vertices per thread per round, their row reads interleaved
    int tb, te;
    share_range(b, P, ntiles, &tb, &te);
    const int qbase = tb * kGrain;
    const int v1 = (int)min((int64_t)te * kGrain, (int64_t)p.n);
    const uint32_t* fb = p.fbits[l & 1];
    int* s_hard = lds;                     // (v, rs, d) triples, kBU per thread at most
    int* s_red = lds + 3 * kBU * kBlock;   // kWaves + 1 ints
    int* s_nh = s_red + kWaves + 1;
    int* s_cnt = s_nh + 1;
    int* s_esum = s_cnt + 1;
    if (threadIdx.x == 0) {
        *s_nh = 0;
        *s_cnt = 0;
        *s_esum = 0;
    }
    lds_barrier();
    int my_e = 0;  // degrees of the vertices this thread settles
    for (int base = tb * kGrain; base < v1; base += kBU * kBlock) {
        int v[kBU], rs[kBU], d[kBU], found[kBU];
#pragma unroll
        for (int i = 0; i < kBU; ++i) {
            v[i] = base + i * kBlock + threadIdx.x;
            rs[i] = d[i] = 0;
            found[i] = -1;
            if (v[i] < v1 && !((p.bitmap[v[i] >> 5] >> (v[i] & 31)) & 1u)) {
                rs[i] = p.offsets[v[i]];
                d[i] = p.offsets[v[i] + 1] - rs[i];
            }
        }
        // the first four neighbours of every row at once
        int c[kBU][4];
#pragma unroll
        for (int i = 0; i < kBU; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) c[i][q] = q < d[i] ? p.cols[rs[i] + q] : -1;
#pragma unroll
        for (int i = 0; i < kBU; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (found[i] < 0 && (unsigned)c[i][q] < (unsigned)p.n && frontier_bit(fb, c[i][q])) found[i] = c[i][q];
        // the next kPullScan neighbours of rows still open, four at a time
        bool hard[kBU];
#pragma unroll
        for (int i = 0; i < kBU; ++i) {
            hard[i] = false;
            if (found[i] < 0 && d[i] > 4) {
                const int f = first_parent_lane(p, rs[i] + 4, d[i] - 4, l, fb);
                if (f >= 0) found[i] = f;
                hard[i] = f == -2;
            }
        }
#pragma unroll
        for (int i = 0; i < kBU; ++i) {
            bu_settle(p, l, qbase, s_cnt, v[i], found[i], found[i] >= 0, true);
            if (found[i] >= 0) my_e += d[i];
            if (hard[i]) {
                const int h = atomicAdd(s_nh, 1);
                s_hard[3 * h] = v[i];
                s_hard[3 * h + 1] = rs[i];
                s_hard[3 * h + 2] = d[i];
            }
        }
        lds_barrier();
        const int nh = *s_nh;
        for (int h = 0; h < nh; ++h) {
            const int hv = s_hard[3 * h], hrs = s_hard[3 * h + 1], hd = s_hard[3 * h + 2];
            const int f = first_hit_wg(p, hrs, hd, [&](int cc) { return frontier_bit(fb, cc); }, s_red);
            bu_settle(p, l, qbase, s_cnt, hv, f, threadIdx.x == 0 && f >= 0, false);
            if (threadIdx.x == 0 && f >= 0) my_e += hd;
        }
        lds_barrier();
        if (threadIdx.x == 0) *s_nh = 0;
        lds_barrier();
    }
    const int we = wave_incl_scan(my_e);
    if (lane_id() == 63 && we) atomicAdd(s_esum, we);
    lds_barrier();
    if (threadIdx.x == 0) {
        p.cnt[b] = *s_cnt;
        p.cnt[p.max_tiles + b] = *s_esum;
    }
    lds_barrier();
}

// ---- a stretch of small levels run by a group of workgroups ---------------------------------
// While a level has at most kSmallN frontier vertices and at most min(small_edges, kGroupCap)
// edges, the first G workgroups of the grid (the group) run it and the rest of the grid waits at
// the next grid barrier: the paper's P_l = min(P, W_l) with P_l small, and one barrier of the
// group per level.  Each target is claimed by a compare-and-swap of its level from -1 to l + 1,
// with its row offsets read alongside: exactly one edge claims each new vertex, so no
// de-duplication pass is needed.  A claim that finds l + 1 is another edge into a vertex of this
// level: with parents, every such edge pushes its source (atomic minimum).
//
// The claiming member keeps each new vertex (id, row start, degree) in its own LDS, and the
// level's totals (entries, edges, vertices reached, the largest member's edges, LDS overflow) add
// up in counters read after the barrier.  When the members' shares of the next level's edges are
// even, each member expands the vertices it claimed (no exchange at all); otherwise every member
// writes its claims to global entry arrays, the group meets once more, and every member stages
// all entries in LDS, takes their exclusive degree sums (the Parallel-Prefix-Sum) and scans an
// equal share [r e / G, (r + 1) e / G) of the edges (Find-StartExpPoint by the wave-row owner
// search).  Entered at level l with the frontier in the parity-l arrays (f_v, f_rs, f_ex); leaves
// with the frontier of level ctrl->resume there.  New vertices get their visited bits (which only
// the levels on the whole grid test) from the member expanding them.
constexpr int kLocalCap = 2048;   // claims a member keeps in LDS per level
constexpr int kLdsNext = 3 * kSmallN + 1;   // LDS offset of the members' claims (v | rs | d)
static_assert(kLdsNext + 3 * kLocalCap + 2 * kWaves + 8 <= kLdsWords, "claims fit in LDS");

// Barrier generations (monotone within a launch): a lite level l uses 4l + 5 and 4l + 6; a
// group level l its exchange 4l + 4 and its end 4l + 7.
__device__ __forceinline__ unsigned long long gen_lite(int l, int k) { return 4ull * l + 4 + k; }
__device__ __forceinline__ unsigned long long gen_exchange(int l) { return 4ull * l + 4; }
__device__ __forceinline__ unsigned long long gen_group_end(int l) { return 4ull * l + 7; }

__device__ __forceinline__ void group_handover(const Params& p, int l, int n, int e_l, int kept, int done, int G,
                                               int rank, int* lds) {
    // every entry of level l is in the global entry arrays: every member scans all degrees in
    // chunks and writes the frontier arrays, and the visited bits, of its own range (the levels
    // on the whole grid need the bits of every vertex reached so far)
    const int par = l & 1;
    int* s_wave = lds_wave(lds);
    const int a = (int)(((int64_t)rank * n) / G), b = (int)(((int64_t)(rank + 1) * n) / G);
    const int32_t* gd = p.aux->gd[par];
    int run = 0;
    for (int c0 = 0; c0 < n; c0 += kBlock * kVTS) {
        int d[kVTS], ts = 0;
        const int i0 = c0 + (int)threadIdx.x * kVTS;
#pragma unroll
        for (int k = 0; k < kVTS; ++k) {
            d[k] = i0 + k < n ? gd[i0 + k] : 0;
            ts += d[k];
        }
        int S;
        int e = run + block_excl_scan(ts, s_wave, &S);
#pragma unroll
        for (int k = 0; k < kVTS; ++k) {
            const int i = i0 + k;
            if (i >= a && i < b) {
                const int v = p.aux->gv[par][i];
                p.f_v[par][i] = v;
                p.f_rs[par][i] = p.aux->grs[par][i];
                p.f_ex[par][i] = e;
                scatter_starts(p, p.tstart[par], i, e, d[k]);
                if ((unsigned)v < (unsigned)p.n)
                    __hip_atomic_fetch_or(&p.bitmap[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                else
                    flag_internal(p.ctrl);
            }
            e += d[k];
        }
        run += S;
    }
    if (rank == 0 && threadIdx.x == 0) {
        if (n <= p.n) p.f_ex[par][n] = e_l;
        else flag_internal(p.ctrl);
        st_rel(&p.ctrl->r_nl, n);
        st_rel(&p.ctrl->r_el, e_l);
        st_rel(&p.ctrl->r_kept, kept);
        st_rel(&p.ctrl->resume, l);
        __hip_atomic_fetch_add(&p.ctrl->small_levels, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

__device__ void group_levels(const Params& p, int l, int n_l, int e_l, int kept, int G, int rank, XGroup& xg,
                             int* lds) {
    int* s_v = lds;                        // frontier being expanded: ids
    int* s_rs = lds + kSmallN;             // row starts
    int* s_ex = lds + 2 * kSmallN;         // exclusive degree sums (+ total)
    int* s_nv = lds + kLdsNext;            // this member's claims: ids
    int* s_nrs = s_nv + kLocalCap;         // row starts
    int* s_nd = s_nrs + kLocalCap;         // degrees
    int* s_wave = lds_wave(lds);
    int* s_wave2 = lds_wave2(lds);
    int* s_misc = lds_misc(lds);           // [0] claims this level, [1] global base, [2..4] totals
    int* s_flag = lds + kLdsWords - 1;
    Ctrl* c = p.ctrl;
    const int cap = min(p.aux->small_edges, kGroupCap);
    bool first = true;
    int done = 0;
    int mine = 0;                          // claims of the previous level kept in LDS
    for (;;) {
        const int par = l & 1, np = (l + 1) & 1;
        // the counters of the frontier two levels back are used again by the next level
        if (rank == 0 && threadIdx.x == 0) {
            const int k = (l + 2) % 3;
            st_rel(&c->g_ne[k], 0ull);
            st_rel(&c->g_rs[k], 0ull);
            st_rel(&c->g_mx[k], 0ull);
            st_rel(&c->g_pos[k], 0ull);
        }
        int n, nloc, g0, g1;
        if (first) {
            // the level the grid handed over: entries with their exclusive sums in f_*[par]
            n = nloc = n_l;
            for (int i = threadIdx.x; i < n; i += kBlock) {
                s_v[i] = p.f_v[par][i];
                s_rs[i] = p.f_rs[par][i];
                s_ex[i] = p.f_ex[par][i];
            }
            if (threadIdx.x == 0) s_ex[n] = e_l;
            __syncthreads();
            g0 = (int)(((int64_t)rank * e_l) / G);
            g1 = (int)(((int64_t)(rank + 1) * e_l) / G);
        } else {
            const unsigned long long ne = ld_acq(&c->g_ne[l % 3]);
            const unsigned long long rs = ld_acq(&c->g_rs[l % 3]);
            const unsigned long long mx = ld_acq(&c->g_mx[l % 3]);
            n = (int)(ne & 0xffffffffull);
            e_l = (int)(ne >> 32);
            kept = (int)(rs >> 32);
            const int spilled = (int)(rs & 0xffffffffull);
            if (rank == 0 && threadIdx.x == 0) {
                if (l < kStatCap && kept > 0) {
                    p.aux->stat_nl[l] = kept;
                    p.aux->stat_el[l] = e_l;
                }
                if (kept > 0) st_rel(&c->levels, l + 1);
                st_rel(&c->heartbeat, l);
            }
            const bool leave = n == 0 || n > kSmallN || e_l > cap;
            // the members' own claims are expanded where they are when no member holds more than
            // half again the average share of the level's edges (or a few hundred edges at all)
            const int64_t avg = (int64_t)e_l / G;
            const bool local = !leave && spilled == 0 && (int64_t)mx <= avg + avg / 2 + 128;
            if (!local && n > 0) {
                // every member's claims go to the global entry arrays, behind those that spilled
                if (threadIdx.x == 0)
                    s_misc[1] = mine ? (int)__hip_atomic_fetch_add(&c->g_pos[l % 3], (unsigned long long)mine,
                                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                     : 0;
                __syncthreads();
                const int base = s_misc[1];
                for (int i = threadIdx.x; i < mine; i += kBlock) {
                    if (base + i < kGroupCap) {
                        p.aux->gv[par][base + i] = s_nv[i];
                        p.aux->grs[par][base + i] = s_nrs[i];
                        p.aux->gd[par][base + i] = s_nd[i];
                    } else {
                        flag_internal(c);
                    }
                }
                if (!sub_barrier(c, p.aux->xbar, xg.xcd, gen_exchange(l), G, true, p.spin_ticks, s_flag)) return;
            }
            if (leave) {
                group_handover(p, l, n, e_l, kept, done, G, rank, lds);
                return;
            }
            if (local) {
                // this member's own claims become its frontier
                nloc = mine;
                int d[kVTS / 2], ts = 0;
                const int i0 = (int)threadIdx.x * (kVTS / 2);
                static_assert(kBlock * (kVTS / 2) == kLocalCap, "thread t moves claims [4t, 4t + 4)");
#pragma unroll
                for (int k = 0; k < kVTS / 2; ++k) {
                    const int i = i0 + k;
                    d[k] = 0;
                    if (i < nloc) {
                        s_v[i] = s_nv[i];
                        s_rs[i] = s_nrs[i];
                        d[k] = s_nd[i];
                    }
                    ts += d[k];
                }
                int S;
                int e = block_excl_scan(ts, s_wave, &S);
#pragma unroll
                for (int k = 0; k < kVTS / 2; ++k) {
                    if (i0 + k < nloc) s_ex[i0 + k] = e;
                    e += d[k];
                }
                if (threadIdx.x == 0) s_ex[nloc] = S;
                g0 = 0;
                g1 = S;
            } else {
                // all entries, from the global arrays
                nloc = n;
                static_assert(kBlock * kVTS == kSmallN, "thread t stages entries [t kVTS, (t + 1) kVTS)");
                int d[kVTS], ts = 0;
                const int i0 = (int)threadIdx.x * kVTS;
#pragma unroll
                for (int k = 0; k < kVTS; ++k) {
                    const int i = i0 + k;
                    d[k] = 0;
                    if (i < n) {
                        s_v[i] = p.aux->gv[par][i];
                        s_rs[i] = p.aux->grs[par][i];
                        d[k] = p.aux->gd[par][i];
                    }
                    ts += d[k];
                }
                int S;
                int e = block_excl_scan(ts, s_wave, &S);
#pragma unroll
                for (int k = 0; k < kVTS; ++k) {
                    if (i0 + k < n) s_ex[i0 + k] = e;
                    e += d[k];
                }
                if (threadIdx.x == 0) s_ex[n] = S;
                g0 = (int)(((int64_t)rank * S) / G);
                g1 = (int)(((int64_t)(rank + 1) * S) / G);
            }
            __syncthreads();
            // visited bits of the entries this member expands (local) or of its share (global)
            const int a = local ? 0 : (int)(((int64_t)rank * n) / G);
            const int b = local ? nloc : (int)(((int64_t)(rank + 1) * n) / G);
            for (int i = a + (int)threadIdx.x; i < b; i += kBlock) {
                const int v = s_v[i];
                if ((unsigned)v < (unsigned)p.n)
                    __hip_atomic_fetch_or(&p.bitmap[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (rank == 0 && threadIdx.x == 0 && l < kStatCap) p.aux->stat_ts[3 * l] = now_ticks();
        if (threadIdx.x == 0) s_misc[0] = 0;
        lds_barrier();
        // expand this member's edges [g0, g1) of its staged entries [0, nloc)
        int my_e = 0, my_r = 0;
        for (int base0 = g0; base0 < g1; base0 += kBlock * kVTS) {
            int own[kVTS];
            static_assert(kVTS == 2 * kVT, "two calls of the row search cover a round");
            owners_of_rows(s_ex, nloc, base0, own);
            owners_of_rows(s_ex, nloc, base0 + kVT * kBlock, own + kVT);
            int v[kVTS], u[kVTS];
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                const int g = base0 + i * kBlock + threadIdx.x;
                v[i] = -1;
                u[i] = -1;
                if (g < g1) {
                    const int lo = own[i];
                    u[i] = s_v[lo];
                    const int idx = s_rs[lo] + (g - s_ex[lo]);
                    if ((unsigned)idx < (unsigned)p.m) {
                        v[i] = p.cols[idx];
                        if ((unsigned)v[i] >= (unsigned)p.n) v[i] = -1;
                    } else {
                        flag_internal(c);
                    }
                }
            }
            // claims, with the claimed rows' offsets read while they are in flight (a visited-
            // bitmap test in front of them cost a round trip more than the claims it saved)
            int old[kVTS], rs[kVTS], re[kVTS];
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                old[i] = -2;
                rs[i] = re[i] = 0;
                if (v[i] >= 0) {
                    int expect = -1;
                    __hip_atomic_compare_exchange_strong(&p.level[v[i]], &expect, l + 1, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    old[i] = expect;
                    rs[i] = p.offsets[v[i]];
                    re[i] = p.offsets[v[i] + 1];
                }
            }
            if (p.parent) {
#pragma unroll
                for (int i = 0; i < kVTS; ++i)
                    if (old[i] == -1 || old[i] == l + 1) parent_push(p, v[i], u[i]);
            }
            // the new vertices with an edge go to this member's LDS, slots reserved per wave;
            // past kLocalCap they spill to the global entry arrays
            int slot[kVTS];
            int wt = 0;
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                const bool fresh = old[i] == -1;
                const uint64_t bb = ballot(fresh && re[i] > rs[i]);
                slot[i] = wt + mbcnt(bb);
                wt += __popcll(bb);
                my_r += fresh ? 1 : 0;
                my_e += fresh ? re[i] - rs[i] : 0;
            }
            int wbase = 0, gbase = 0;
            if (lane_id() == 0 && wt) {
                wbase = atomicAdd(&s_misc[0], wt);
                const int sp = wbase + wt - max(wbase, kLocalCap);
                if (sp > 0)
                    gbase = (int)__hip_atomic_fetch_add(&c->g_pos[(l + 1) % 3], (unsigned long long)sp,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            wbase = __shfl(wbase, 0);
            gbase = __shfl(gbase, 0);
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                if (old[i] == -1 && re[i] > rs[i]) {
                    const int s = wbase + slot[i];
                    if (s < kLocalCap) {
                        s_nv[s] = v[i];
                        s_nrs[s] = rs[i];
                        s_nd[s] = re[i] - rs[i];
                    } else {
                        const int gs = gbase + s - max(wbase, kLocalCap);
                        if (gs < kGroupCap) {
                            p.aux->gv[np][gs] = v[i];
                            p.aux->grs[np][gs] = rs[i];
                            p.aux->gd[np][gs] = re[i] - rs[i];
                        } else {
                            flag_internal(c);
                        }
                    }
                }
            }
        }
        // the member's totals for the next level
        {
            const int we = wave_incl_scan(my_e), wr = wave_incl_scan(my_r);
            if (lane_id() == 63) {
                s_wave[wave_id()] = we;
                s_wave2[wave_id()] = wr;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int te = 0, tr = 0;
#pragma unroll
                for (int q = 0; q < kWaves; ++q) {
                    te += s_wave[q];
                    tr += s_wave2[q];
                }
                const int claims = s_misc[0];
                const int sp = max(claims - kLocalCap, 0);
                const int k = (l + 1) % 3;
                if (claims)
                    __hip_atomic_fetch_add(&c->g_ne[k], ((unsigned long long)te << 32) | (unsigned)claims,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (tr || sp)
                    __hip_atomic_fetch_add(&c->g_rs[k], ((unsigned long long)tr << 32) | (unsigned)sp,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (te) __hip_atomic_fetch_max(&c->g_mx[k], (unsigned long long)te, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                s_misc[2] = min(claims, kLocalCap);
                s_misc[3] = sp;
            }
            __syncthreads();
            mine = s_misc[2];
        }
        if (rank == 0 && threadIdx.x == 0 && l < kStatCap) p.aux->stat_ts[3 * l + 1] = now_ticks();
        // only claims that spilled to the global entry arrays are plain stores other members read
        if (!sub_barrier(c, p.aux->xbar, xg.xcd, gen_group_end(l), G, true, p.spin_ticks, s_flag, s_misc[3] > 0)) return;
        if (rank == 0 && threadIdx.x == 0 && l < kStatCap) p.aux->stat_ts[3 * l + 2] = now_ticks();
        ++l;
        ++done;
        first = false;
    }
}

// ---- parent pass (plain per-level comparator only) -------------------------------------------
// parent[v] = smallest-id neighbour one level closer (rows are sorted, so the
// first such neighbour in the row), parent[root] = root, -1 if unreached.
__device__ void parent_range(const Params& p, int64_t first, int64_t stride) {
    for (int64_t v = first; v < p.n; v += stride) {
        const int lv = p.level[v];
        int par = -1;
        if (lv == 0) {
            par = (int)v;
        } else if (lv > 0) {
            const int e0 = p.offsets[v], e1 = p.offsets[v + 1];
            for (int e = e0; e < e1; ++e) {
                const int u = p.cols[e];
                if (p.level[u] == lv - 1) { par = u; break; }
            }
        }
        p.parent[v] = par;
    }
}

// ---- kernels ---------------------------------------------------------------------------------

// Resets the control block and the per-run arrays: level = -1, parent = -1
// (all bits set, so unsigned minima replace it), bitmap = 0, and the
// descriptors of the roots' compaction.
__global__ void __launch_bounds__(kBlock) k_prep(Params p, int prep_shares, int fill_parent) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < p.n; v += stride) {
        p.level[v] = -1;
        if (fill_parent) p.parent[v] = -1;
    }
    const int64_t words = ((int64_t)p.n + 31) >> 5;
    for (int64_t w = tid; w < words; w += stride) p.bitmap[w] = 0u;
    for (int64_t w = tid; w < p.hot_words; w += stride) p.hot[0][w] = p.hot[1][w] = 0u;
    if (p.direction || p.fb_pull || p.dense_edges > 0)
        for (int64_t w = tid; w < words; w += stride) p.fbits[0][w] = p.fbits[1][w] = 0u;
    for (int64_t t = tid; t < prep_shares; t += stride) p.desc[1][t] = 0ull;
    constexpr int64_t xwords = sizeof(XBar) / sizeof(unsigned long long);
    for (int64_t w = tid; w < xwords; w += stride) reinterpret_cast<unsigned long long*>(p.xbar)[w] = 0ull;
    if (tid == 0) {
        Aux* a = p.aux;
        a->stat_nl = p.stat_nl;
        a->stat_el = p.stat_el;
        a->stat_ts = p.stat_ts;
        a->roots = p.roots;
        a->xbar = p.xbar;
        a->snap = p.snap;
        for (int k = 0; k < 2; ++k) {
            a->gv[k] = p.gv[k];
            a->grs[k] = p.grs[k];
            a->gd[k] = p.gd[k];
        }
        a->small_edges = p.small_edges;
        a->bu_alpha = p.bu_alpha;
        a->bu_beta = p.bu_beta;
        a->insensitive = p.insensitive;
        a->group = p.group;
        Ctrl* c = p.ctrl;
        c->bar = 0;
        c->nl[0] = c->nl[1] = 0;
        c->el[0] = c->el[1] = 0;
        c->kept[0] = c->kept[1] = 0;
        c->levels = 0;
        c->error = 0;
        c->small_levels = 0;
        c->resume = 0;
        c->heartbeat = 0;
        c->plain_next = 0;
        c->r_nl = c->r_el = c->r_kept = 0;
        c->bu_levels = 0;
        for (int k = 0; k < 3; ++k) c->g_ne[k] = c->g_rs[k] = c->g_mx[k] = c->g_pos[k] = 0ull;
    }
}

// Gives the frontier, start-point, queue and descriptor arrays of a search's
// scratch defined contents (zeros; owner = -1 for "no slot"), as a freshly
// created workspace has them, so that nothing left by an earlier search of
// another graph in the same memory can hold an out-of-range index.
__global__ void __launch_bounds__(kBlock) k_scrub(Params p) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nv = (int64_t)p.n + 2;
    for (int64_t i = tid; i < nv; i += stride) {
#pragma unroll
        for (int k = 0; k < 2; ++k) p.f_v[k][i] = p.f_rs[k][i] = p.f_ex[k][i] = 0;
    }
    for (int64_t i = tid; i < p.n; i += stride) p.owner[i] = -1;
    for (int64_t t = tid; t < p.max_tiles; t += stride) {
        p.tstart[0][t] = p.tstart[1][t] = 0;
        p.desc[0][t] = p.desc[1][t] = 0ull;
        p.cnt[t] = p.cnt[p.max_tiles + t] = 0;
    }
    for (int64_t i = tid; i < p.cand_cap; i += stride) p.cand[i] = 0;
}

// Device status of the search that ran before it on the stream: BFS_OK, or
// BFS_EDEVICE if a wait of the level loop timed out or found an inconsistency.
__global__ void k_status(const Ctrl* c, int32_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = c->error == 0 ? 0 : BFS_EDEVICE_CODE;
}

// Roots become the private queues of level -1: root i sits in slot i, and
// share b of the roots' P_r shares owns slots [tb * kGrain, te * kGrain).
__device__ void roots_range(const Params& p, int P, int64_t first, int64_t stride) {
    const int rtiles = (p.nroots + kGrain - 1) / kGrain;
    for (int64_t i = first; i < p.nroots; i += stride) {
        const int r = p.aux->roots ? p.aux->roots[i] : p.single_root;
        p.level[r] = 0;
        if (p.parent) p.parent[r] = r;
        p.owner[r] = (int)i;
        p.cand[i] = r;
    }
    for (int64_t b = first; b < P; b += stride) {
        int tb, te;
        share_range((int)b, P, rtiles, &tb, &te);
        p.cnt[b] = (int)max((int64_t)0, min((int64_t)te * kGrain, (int64_t)p.nroots) - (int64_t)tb * kGrain);
    }
}

// hot[w] bit j = visited bit of the vertex with hot number 32 w + j (0 past
// hot_count), 64 hot numbers per wave step: the hot bits of levels <= l when
// the visited bitmap holds exactly the vertices of levels <= l.
__device__ __forceinline__ void rebuild_hot_bits(const Params& p, uint32_t* hot, int64_t first, int64_t stride) {
    const int64_t nh = (int64_t)p.hot_words * 32;
    for (int64_t h0 = first - lane_id(); h0 < nh; h0 += stride) {  // wave-uniform base, a multiple of 64
        const int64_t h = h0 + lane_id();
        bool bit = false;
        if (h < p.hot_count) {
            const int v = p.hot_vid[h];
            bit = (unsigned)v < (unsigned)p.n && ((p.bitmap[v >> 5] >> (v & 31)) & 1u);
        }
        const uint64_t bb = ballot(bit);
        if ((lane_id() & 31) == 0 && h < nh) hot[h >> 5] = (uint32_t)(bb >> (lane_id() & 32));
    }
}

// After a dense level's expansion: its hot discoveries, hot[next] & ~hot[cur]
// (the current bits are exact on dense levels), get the visited bits the
// expansion left unset, so that the compaction finds them among the bits
// set since the level's snapshot.  Grid-strided over the hot words.
__device__ __forceinline__ void merge_hot_discoveries(const Params& p, const uint32_t* hcur, const uint32_t* hnext,
                                                      int64_t first, int64_t stride) {
    for (int64_t w = first; w < p.hot_words; w += stride) {
        uint32_t x = hnext[w] & ~hcur[w];
        while (x) {
            const int64_t h = w * 32 + __builtin_ctz(x);
            x &= x - 1;
            if (h < p.hot_count) {
                const int v = p.hot_vid[h];
                if ((unsigned)v < (unsigned)p.n)
                    __hip_atomic_fetch_or(&p.bitmap[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

__device__ __forceinline__ int shares_for(int ntiles, int G) { return ntiles < G ? ntiles : G; }

// Register budget of the persistent kernel: its occupancy (workgroups per
// CU) is what hides the memory latency of the level loop.
#ifndef BFS_PERSISTENT_WAVES_PER_EU
#define BFS_PERSISTENT_WAVES_PER_EU 4
#endif
// DIR: bottom-up levels are possible (BFS_MODE_DIRECTION).  The two variants
// are separate kernels so that the top-down one keeps its own register budget.
template <bool DIR>
__global__ void __attribute__((amdgpu_waves_per_eu(BFS_PERSISTENT_WAVES_PER_EU))) __launch_bounds__(kBlock)
k_persistent(Params p) {
    __shared__ Lds lds_s;
    int* lds = lds_s.w;
    int* s_flag = lds + kLdsWords - 1;
    const int G = gridDim.x;
    Ctrl* c = p.ctrl;

    const int rtiles = (p.nroots + kGrain - 1) / kGrain;
    const int Pr = shares_for(rtiles, G);
    [[clang::always_inline]] roots_range(p, Pr, (int64_t)blockIdx.x * kBlock + threadIdx.x, (int64_t)G * kBlock);
    // the first barrier is the flat one; it also counts the workgroups on each XCD
    XGroup xg{0, 1, 1};
    if (threadIdx.x == 0) xbar_join(p.aux->xbar, xcd_id());
    if (!grid_barrier(c, p.spin_ticks, s_flag)) return;
    if (threadIdx.x == 0) xg = xbar_group(p.aux->xbar, xcd_id());
    bool ok = true;
    if (blockIdx.x < Pr) {
        [[clang::always_inline]] ok = compact_share(p, -1, blockIdx.x, Pr, rtiles, false, true, lds);
    }
    if (!ok) return;
    if (!xcd_barrier(c, p.aux->xbar, xg, p.spin_ticks, s_flag)) return;

    // The size of each level is read once, right after the barrier that
    // publishes it, into loop-carried values: the slot it came from may be
    // rewritten before every workgroup would otherwise have read it again.
    int l = 0;
    int n_l = ld_acq(&c->nl[0]);
    int e_l = ld_acq(&c->el[0]);
    int kept = ld_acq(&c->kept[0]);
    // direction optimisation: fbits[l & 1] is exact when level l - 1 went through
    // compact_share (the roots do); edges of vertices reached so far, for the switch rule
    bool fbits_ok = true, bottom_up = false;
    // hot[l & 1] holds exactly the hot vertices visited up to level l: the expansion keeps
    // it so once it is, but the roots and group levels set no hot bits
    bool hot_ok = false;
    // top-down loop: fbits[x] holds bits a later writer must clear first
    bool fb_dirty[2] = {p.fb_pull != 0, false};
    int64_t reached_edges = 0;
    const int fwords = (p.n + 31) >> 5;
    for (;;) {
        const int par = l & 1;
        const bool rec = blockIdx.x == 0 && threadIdx.x == 0 && l < kStatCap;
        if (rec) p.aux->stat_ts[3 * l] = now_ticks();
        if (blockIdx.x == 0 && threadIdx.x == 0 && kept > 0) {
            if (l < kStatCap) { p.aux->stat_nl[l] = kept; p.aux->stat_el[l] = e_l; }
            st_rel(&c->levels, l + 1);
        }
        if (n_l == 0) break;
        reached_edges += e_l;
        if (p.aux->small_edges > 0 && n_l <= kSmallN && e_l <= min(p.aux->small_edges, kGroupCap)) {
            const int Gs = max(1, min(p.aux->group, G));
            if ((int)blockIdx.x < Gs) {
                [[clang::always_inline]] group_levels(p, l, n_l, e_l, kept, Gs, blockIdx.x, xg, lds);
            }
            if (!xcd_barrier(c, p.aux->xbar, xg, p.spin_ticks, s_flag)) return;
            // every member has read the append counters: the next stretch, at least one grid
            // level away, starts from zero
            if (blockIdx.x == 0 && threadIdx.x == 0)
                for (int k = 0; k < 3; ++k) {
                    st_rel(&c->g_ne[k], 0ull);
                    st_rel(&c->g_rs[k], 0ull);
                    st_rel(&c->g_mx[k], 0ull);
                    st_rel(&c->g_pos[k], 0ull);
                }
            l = ld_acq(&c->resume);
            n_l = ld_acq(&c->r_nl);
            e_l = ld_acq(&c->r_el);
            kept = ld_acq(&c->r_kept);
            fbits_ok = false;  // group levels keep no frontier or hot bits
            hot_ok = false;
            bottom_up = false;
            // Direction mode: when the level the group hands over is one that Beamer's rule
            // sends bottom-up, its frontier bits are rebuilt from the handed-over queue (the
            // other buffer cleared), rather than expanding it top-down over its hubs
            if (DIR && n_l > 0 && !(n_l <= kSmallN && e_l <= min(p.aux->small_edges, kGroupCap)) &&
                (int64_t)e_l * p.aux->bu_alpha > p.m - reached_edges - e_l) {
                for (int w = blockIdx.x * kBlock + threadIdx.x; w < fwords; w += G * kBlock) {
                    p.fbits[0][w] = 0u;
                    p.fbits[1][w] = 0u;
                }
                if (!xcd_barrier(c, p.aux->xbar, xg, p.spin_ticks, s_flag)) return;
                const int32_t* fv = p.f_v[l & 1];
                uint32_t* fb = p.fbits[l & 1];
                for (int i = blockIdx.x * kBlock + threadIdx.x; i < n_l; i += G * kBlock) {
                    const int v = fv[i];
                    if ((unsigned)v < (unsigned)p.n)
                        __hip_atomic_fetch_or(&fb[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                }
                if (!xcd_barrier(c, p.aux->xbar, xg, p.spin_ticks, s_flag)) return;
                fbits_ok = true;
            }
            continue;
        }
        // Beamer's rule: go bottom-up once the frontier's edges outweigh those of the
        // unreached vertices (by alpha), return when the frontier is small (by beta)
        if (DIR) {
            const int64_t unreached = p.m - reached_edges;
            bottom_up = fbits_ok && (bottom_up ? (int64_t)n_l * p.aux->bu_beta >= p.n
                                               : (int64_t)e_l * p.aux->bu_alpha > unreached);
        }
        const int ntiles = bottom_up ? (p.n + kGrain - 1) / kGrain : (int)(((int64_t)e_l + kGrain - 1) / kGrain);
        // P_l = min(P, W_l); the work-insensitive variant splits every level over all P
        // workgroups (one share per look-back descriptor), most of them empty on small levels
        const int P = p.aux->insensitive ? min(G, p.max_tiles) : shares_for(ntiles, G);
        const int np = (l + 1) & 1;
        const bool push = p.parent && e_l <= p.push_edges;
        // a dense level keeps its new frontier as bits and compacts it in vertex order
        const bool dense = !DIR && !push && p.dense_edges > 0 && e_l >= p.dense_edges;
        const int Pd = dense ? dense_shares(p, G) : 0;
        // A lite level (few workgroups, not dense) skips the upkeep that only pays on large
        // levels: it merges no hot bits and keeps no frontier bits for the next level's pulls
        const bool lite = !DIR && !dense && P < kLiteShares;
        const bool keep_fb = !DIR && p.fb_pull && !lite;  // this level's compaction keeps frontier bits
        // the host sizes the private queues for every level its options let keep them; a level
        // beyond that (which it never launches) stops the run with an error instead of writing past
        if (!dense && !(DIR && bottom_up) && (int64_t)ntiles * kGrain > p.cand_cap) {
            if (blockIdx.x == 0 && threadIdx.x == 0) flag_internal(c);
            return;  // every workgroup takes this branch at the same level
        }
        // reset this level's compaction state (last used two levels ago)
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st_rel(&c->kept[np], 0);
            if (bottom_up) c->bu_levels += 1;
        }
        for (int t = blockIdx.x * kBlock + threadIdx.x; t < max(P, Pd); t += G * kBlock) p.desc[par][t] = 0ull;
        // Frontier bits.  Direction mode: fbits[np] is zero when a level starts (its own
        // level cleared it after reading it), except right after a stretch of
        // group levels, which keep none; that level runs top-down, so nothing
        // writes fbits[np] before its compaction and it can be cleared now.  Top-down
        // loop: the previous level's pulls were the last readers of fbits[np], and this
        // level's compaction is its first writer; a level that writes none leaves the buffer
        // as it is.  A dense level's compaction overwrites every word of fbits[np], and its
        // expansion waits at an extra barrier for the snapshot of the visited bits.
        const bool fb_write = !DIR && (keep_fb || dense);
        if ((DIR && !fbits_ok) || (!dense && fb_write && fb_dirty[np]))
            for (int w = blockIdx.x * kBlock + threadIdx.x; w < fwords; w += G * kBlock) p.fbits[np][w] = 0u;
        if (dense)  // the visited bits before the level; the compaction writes every word of fbits[np]
            for (int w = blockIdx.x * kBlock + threadIdx.x; w < fwords; w += G * kBlock) p.aux->snap[w] = p.bitmap[w];
        if (fb_write) fb_dirty[np] = true;
        // A dense level drops a hot target only by its hot bits; where those miss visited
        // vertices (the roots and group levels set none), each such edge would
        // set a visited bit again, which the snapshot then does not count as new, so the
        // bits are rebuilt here from the visited bitmap (exactly the vertices of levels <= l)
        if (dense && p.hot_words > 0 && !hot_ok) {
            rebuild_hot_bits(p, p.hot[par], blockIdx.x * kBlock + threadIdx.x, G * kBlock);
            hot_ok = true;
        }
        if (dense && !xcd_barrier(c, p.aux->xbar, xg, p.spin_ticks, s_flag)) return;
        if (DIR && bottom_up) {
            if (blockIdx.x < P) bottom_up_share(p, l, blockIdx.x, P, ntiles, lds);
        } else if (blockIdx.x < P) {
            if (p.split_search) search_starts(p, l, blockIdx.x, P, ntiles, n_l);
            [[clang::always_inline]] expand_share(p, l, blockIdx.x, P, ntiles, n_l, e_l, lds, dense, lite);
        }
        // a lite level's compaction needs only its own workgroups' expansion, so only they
        // meet here; the others wait for the level's end
        if (lite) {
            if (blockIdx.x < P && !sub_barrier(c, p.aux->xbar, xg.xcd, gen_lite(l, 1), P, true, p.spin_ticks, s_flag))
                return;
            hot_ok = false;
        } else if (!xcd_barrier(c, p.aux->xbar, xg, p.spin_ticks, s_flag)) {
            return;
        }
        if (dense && p.hot_words > 0) {
            merge_hot_discoveries(p, p.hot[par], p.hot[np], (int64_t)blockIdx.x * kBlock + threadIdx.x,
                                  (int64_t)G * kBlock);
            if (!xcd_barrier(c, p.aux->xbar, xg, p.spin_ticks, s_flag)) return;
        }
        if (rec) p.aux->stat_ts[3 * l + 1] = now_ticks();
        if (DIR)  // this level's frontier bits have been read: clear them for level l + 2
            for (int w = blockIdx.x * kBlock + threadIdx.x; w < fwords; w += G * kBlock) p.fbits[par][w] = 0u;
        if (DIR && bottom_up) {
            // next frontier size from the shares' counts; a following bottom-up level
            // needs only the frontier bits, so the queue is linearised only otherwise
            int tn = 0, te_sum = 0;
            for (int j = threadIdx.x; j < P; j += kBlock) {
                tn += p.cnt[j];
                te_sum += p.cnt[p.max_tiles + j];
            }
            int n_next, e_next;
            block_excl_scan(tn, lds_wave(lds), &n_next);
            block_excl_scan(te_sum, lds_wave2(lds), &e_next);
            const bool next_small = p.aux->small_edges > 0 && n_next <= kSmallN && e_next <= min(p.aux->small_edges, kGroupCap);
            if (n_next > 0 && !next_small && (int64_t)n_next * p.aux->bu_beta >= p.n) {
                if (!xcd_barrier(c, p.aux->xbar, xg, p.spin_ticks, s_flag)) return;
                if (rec) p.aux->stat_ts[3 * l + 2] = now_ticks();
                ++l;
                n_l = n_next;
                e_l = e_next;
                kept = n_next;
                fbits_ok = true;
                continue;
            }
            if (blockIdx.x < P) {
                [[clang::always_inline]] ok = compact_share(p, l, blockIdx.x, P, ntiles, false, false, lds, true);
                if (!ok) return;
            }
        } else {
            // pulls test the frontier bits of level l (2 MiB for 2^24 vertices) instead of the
            // level array when they are exact: not right after group levels
            const uint32_t* fpull = (!DIR && p.fb_pull && fbits_ok) ? p.fbits[par] : nullptr;
            if (dense) {
                if (blockIdx.x < Pd) [[clang::always_inline]] ok = dense_compact_share(p, l, blockIdx.x, Pd, lds, fpull);
            } else if (blockIdx.x < P) {
                [[clang::always_inline]] ok =
                    compact_share(p, l, blockIdx.x, P, ntiles, !push, push, lds, false, fpull, keep_fb);
            }
            if (!ok) return;
        }
        fbits_ok = DIR || fb_write;  // top-down: fbits[np] holds exactly the next frontier
        if (lite) {
            if (!sub_barrier(c, p.aux->xbar, xg.xcd, gen_lite(l, 2), P, blockIdx.x < P, p.spin_ticks, s_flag)) return;
        } else if (!xcd_barrier(c, p.aux->xbar, xg, p.spin_ticks, s_flag)) {
            return;
        }
        if (rec) p.aux->stat_ts[3 * l + 2] = now_ticks();
        ++l;
        n_l = ld_acq(&c->nl[np]);
        e_l = ld_acq(&c->el[np]);
        kept = ld_acq(&c->kept[np]);
    }
}

// ---- per-level launches (BFS_MODE_LEVEL) ---------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_level_roots(Params p, int P) {
    roots_range(p, P, (int64_t)blockIdx.x * kBlock + threadIdx.x, (int64_t)gridDim.x * kBlock);
}

// One workgroup per share (grid = P).
__global__ void __launch_bounds__(kBlock) k_level_compact(Params p, int l, int ntiles) {
    __shared__ Lds lds_s;
    const bool push = l < 0 || (p.parent && ld_acq(&p.ctrl->el[l & 1]) <= p.push_edges);
    compact_share(p, l, blockIdx.x, gridDim.x, ntiles, !push, push, lds_s.w);
}

__global__ void __launch_bounds__(kBlock) k_level_expand(Params p, int l, int ntiles) {
    __shared__ Lds lds_s;
    const int n_l = ld_acq(&p.ctrl->nl[l & 1]);
    const int e_l = ld_acq(&p.ctrl->el[l & 1]);
    const int par = l & 1, np = (l + 1) & 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) st_rel(&p.ctrl->kept[np], 0);
    if (threadIdx.x == 0) p.desc[par][blockIdx.x] = 0ull;
    if (p.split_search) search_starts(p, l, blockIdx.x, gridDim.x, ntiles, n_l);
    expand_share(p, l, blockIdx.x, gridDim.x, ntiles, n_l, e_l, lds_s.w);
}

__global__ void __launch_bounds__(kBlock) k_parent(Params p) {
    parent_range(p, (int64_t)blockIdx.x * kBlock + threadIdx.x, (int64_t)gridDim.x * kBlock);
}

// ---- plain per-level kernel (comparator): one thread per frontier vertex -------------------

__global__ void k_plain_init(Params p, int32_t* fv0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        p.level[p.single_root] = 0;
        fv0[0] = p.single_root;
    }
}

__global__ void __launch_bounds__(256) k_plain_level(Params p, int l, const int32_t* fv, int nf, int32_t* fv_next) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int u = fv[i];
    for (int e = p.offsets[u]; e < p.offsets[u + 1]; ++e) {
        const int v = p.cols[e];
        if (p.level[v] == -1 && atomicCAS(&p.level[v], -1, l + 1) == -1) {
            const int pos = atomicAdd(&p.ctrl->plain_next, 1);
            fv_next[pos] = v;
        }
    }
}

// ---- primitive test kernel: compaction of given private queues ------------------------------

__global__ void __launch_bounds__(kBlock) k_prim_compact(Params p, int ntiles) {
    __shared__ Lds lds_s;
    compact_share(p, 0, blockIdx.x, gridDim.x, ntiles, false, true, lds_s.w);
}

__global__ void k_prim_reset(Params p, int P) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t t = tid; t < P; t += (int64_t)gridDim.x * blockDim.x) p.desc[0][t] = 0ull;
    if (tid == 0) {
        p.ctrl->kept[1] = 0;
        p.ctrl->nl[1] = 0;
        p.ctrl->el[1] = 0;
        p.ctrl->error = 0;
    }
}

__global__ void k_prim_totals(Params p, int32_t* totals) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int nl = p.ctrl->nl[1], el = p.ctrl->el[1];
        totals[0] = nl;
        totals[1] = el;
        if (nl >= 0 && nl <= p.n) p.f_ex[1][nl] = el;  // the total after the last entry, also for no entries
    }
}

// ---- host launchers ----------------------------------------------------------------------------

int persistent_grid_capacity(int device) {
    int per_cu = 0, per_cu_dir = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_persistent<false>),
                                                     kBlock, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_dir, reinterpret_cast<const void*>(k_persistent<true>),
                                                     kBlock, 0) != hipSuccess)
        return 0;
    per_cu = per_cu < per_cu_dir ? per_cu : per_cu_dir;  // one grid size serves both variants
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    return per_cu * cus;
}

static int fill_grid(int64_t items) {
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

// Graph set-up for the hot-vertex filter: colx[e] = cols[e], or -1 - its hot
// number for a hot target (INT32_MIN for a target outside [0, n)).
__global__ void k_hot_gather(const int32_t* cols, int64_t m, const int32_t* hidx, int32_t* colx, int32_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        const int32_t v = cols[e];
        int32_t x = INT32_MIN;
        if ((unsigned)v < (unsigned)n) x = hidx[v] >= 0 ? -1 - hidx[v] : v;
        colx[e] = x;
    }
}

hipError_t launch_hot_gather(const int32_t* cols, int64_t m, const int32_t* hidx, int32_t* colx, int32_t n,
                             hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_hot_gather, dim3(fill_grid(m)), dim3(kBlock), 0, s, cols, m, hidx, colx, n);
    return hipGetLastError();
}

hipError_t launch_prep(const Params& p, int prep_shares, bool fill_parent, hipStream_t s) {
    hipLaunchKernelGGL(k_prep, dim3(fill_grid(p.n)), dim3(kBlock), 0, s, p, prep_shares, fill_parent ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_scrub(const Params& p, hipStream_t s) {
    const int64_t items = p.cand_cap > (int64_t)p.n + 2 ? p.cand_cap : (int64_t)p.n + 2;
    hipLaunchKernelGGL(k_scrub, dim3(fill_grid(items)), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_status(const Ctrl* c, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, s, c, out);
    return hipGetLastError();
}

hipError_t launch_persistent(const Params& p, int grid, hipStream_t s) {
    if (p.direction) hipLaunchKernelGGL(k_persistent<true>, dim3(grid), dim3(kBlock), 0, s, p);
    else hipLaunchKernelGGL(k_persistent<false>, dim3(grid), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_level_roots(const Params& p, int shares, hipStream_t s) {
    hipLaunchKernelGGL(k_level_roots, dim3(fill_grid(p.nroots > shares ? p.nroots : shares)), dim3(kBlock), 0, s, p,
                       shares);
    return hipGetLastError();
}

hipError_t launch_level_compact(const Params& p, int l, int ntiles, int shares, hipStream_t s) {
    hipLaunchKernelGGL(k_level_compact, dim3(shares), dim3(kBlock), 0, s, p, l, ntiles);
    return hipGetLastError();
}

hipError_t launch_level_expand(const Params& p, int l, int ntiles, int shares, hipStream_t s) {
    hipLaunchKernelGGL(k_level_expand, dim3(shares), dim3(kBlock), 0, s, p, l, ntiles);
    return hipGetLastError();
}

hipError_t launch_parent(const Params& p, hipStream_t s) {
    hipLaunchKernelGGL(k_parent, dim3(fill_grid(p.n)), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_plain_init(const Params& p, int32_t* fv0, hipStream_t s) {
    hipLaunchKernelGGL(k_plain_init, dim3(1), dim3(64), 0, s, p, fv0);
    return hipGetLastError();
}

hipError_t launch_plain_level(const Params& p, int l, const int32_t* fv, int nf, int32_t* fv_next,
                              hipStream_t s) {
    const int g = (nf + 255) / 256;
    hipLaunchKernelGGL(k_plain_level, dim3(g > 0 ? g : 1), dim3(256), 0, s, p, l, fv, nf, fv_next);
    return hipGetLastError();
}

hipError_t launch_prim_compact(const int32_t* offsets, int32_t n, const int32_t* owner, const int32_t* cand,
                               const int32_t* cnt, int32_t ntiles, int32_t* out_v, int32_t* out_rs, int32_t* out_ex,
                               int32_t* out_tstart, int32_t tstart_cap, int32_t* totals, unsigned long long* desc,
                               Ctrl* ctrl, uint32_t* bitmap, hipStream_t s) {
    // one share per tile: share t's private queue is tile t's
    Params p{};
    p.offsets = offsets;
    p.n = n;
    p.max_tiles = tstart_cap;
    p.cand_cap = (int64_t)ntiles * kGrain;
    p.owner = const_cast<int32_t*>(owner);
    p.cand = const_cast<int32_t*>(cand);
    p.cnt = const_cast<int32_t*>(cnt);
    p.f_v[1] = out_v;
    p.f_rs[1] = out_rs;
    p.f_ex[1] = out_ex;
    p.tstart[1] = out_tstart;
    p.desc[0] = desc;
    p.ctrl = ctrl;
    p.bitmap = bitmap;
    p.spin_ticks = 300000000ull;
    hipLaunchKernelGGL(k_prim_reset, dim3(fill_grid(ntiles)), dim3(kBlock), 0, s, p, ntiles);
    if (ntiles > 0) hipLaunchKernelGGL(k_prim_compact, dim3(ntiles), dim3(kBlock), 0, s, p, ntiles);
    hipLaunchKernelGGL(k_prim_totals, dim3(1), dim3(64), 0, s, p, totals);
    return hipGetLastError();
}

}  // namespace s3bfs
