// HIP kernels of the S3BFS level loop for gfx950 (wave64, CDNA4).
//
// One level of the paper's Figure 1 maps onto two phases:
//
//   expand   Each share of kGrain consecutive frontier edges (a "tile",
//            the paper's per-thread share of e_l) is scanned by one
//            workgroup.  The tile's slice of the frontier's degree prefix
//            sums is staged in LDS; every lane finds the vertex owning its
//            edge by binary search there, reads the neighbour id (coalesced
//            int32 reads of cols), filters it through the visited bitmap and
//            the level array, stores level = l + 1 (every racing writer
//            stores the same value) and owner = its candidate slot, and
//            appends the vertex to the tile's private queue (EXPLORE-VERTEX,
//            with the benign race of the Algorithm paragraph).
//   compact  Each tile's queue keeps the entries whose slot still owns the
//            vertex (Owner de-duplication), reads the survivors' degrees,
//            and a decoupled look-back scan over tiles gives every survivor
//            its position in the next frontier and its exclusive degree sum
//            (the Sizes prefix sum and linearisation fused with the next
//            level's degree gather and Parallel-Prefix-Sum).  Each survivor
//            then writes itself as the start point of every share that
//            begins inside its edge range (Find-StartExpPoint's scatter).
//
// The persistent kernel runs all levels in one launch with a grid barrier
// between phases; only ceil(e_l / kGrain) workgroups have work in a phase
// (P_l = min(P, W_l)), and while a level is small a single workgroup runs
// it alone out of LDS, synchronising with __syncthreads only, so the rest of
// the grid idles (the paper's "no more cores than the work needs").
#include "bfs_internal.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s3bfs {

#define BFS_EDEVICE_CODE (-8)
#define BFS_EINTERNAL_CODE (-9)

// ---- small helpers ---------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

template <typename T>
__device__ __forceinline__ T ld_acq(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_rel(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// Inclusive prefix sum over a full wave (all 64 lanes must be active):
// DPP row shifts scan each row of 16 lanes, then the row totals are added
// from lanes 15, 31 and 47.
__device__ __forceinline__ int wave_incl_scan(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
    const int r0 = __builtin_amdgcn_readlane(x, 15);
    const int r1 = __builtin_amdgcn_readlane(x, 31);
    const int r2 = __builtin_amdgcn_readlane(x, 47);
    const int row = lane_id() >> 4;
    x += (row >= 1 ? r0 : 0) + (row >= 2 ? r1 : 0) + (row >= 3 ? r2 : 0);
    return x;
}

// Exclusive block-wide prefix sum of one int per thread; *total gets the sum.
// s_tmp holds kWaves ints.  Must be called by the whole workgroup.
__device__ __forceinline__ int block_excl_scan(int x, int* s_tmp, int* total) {
    const int incl = wave_incl_scan(x);
    if (lane_id() == 63) s_tmp[wave_id()] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int t = s_tmp[w];
        base += (w < wave_id()) ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + incl - x;
}

__device__ __forceinline__ uint64_t ballot(bool f) { return __builtin_amdgcn_ballot_w64(f); }
__device__ __forceinline__ int mbcnt(uint64_t b) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0));
}

// Waits for `pred` with a time-out that is extended whenever ctrl->heartbeat
// moves.  Returns false (and records BFS_EDEVICE) on time-out or if another
// workgroup already failed.
template <typename Pred>
__device__ bool spin_until(Ctrl* c, uint64_t spin_ticks, Pred pred) {
    uint64_t t0 = now_ticks();
    int hb = ld_acq(&c->heartbeat);
    while (!pred()) {
        __builtin_amdgcn_s_sleep(1);
        if (ld_acq(&c->error) != 0) return false;
        const int hb2 = ld_acq(&c->heartbeat);
        if (hb2 != hb) { hb = hb2; t0 = now_ticks(); }
        if (now_ticks() - t0 > spin_ticks) {
            __hip_atomic_store(&c->error, BFS_EDEVICE_CODE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// Grid-wide barrier for a grid whose workgroups are all resident.  The
// agent-scope release before arriving writes this XCD's dirty L2 lines back
// and the acquire after leaving invalidates stale ones, so every write made
// before the barrier by any workgroup is visible after it on every XCD.
// Returns false on failure; every workgroup then leaves the kernel.
__device__ bool grid_barrier(Ctrl* c, uint64_t spin_ticks, int* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned long long nb = gridDim.x;
        const unsigned long long arrived =
            __hip_atomic_fetch_add(&c->bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long target = (arrived / nb + 1) * nb;
        bool ok = spin_until(c, spin_ticks, [&] { return ld_acq(&c->bar) >= target; });
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_flag = ok && ld_acq(&c->error) == 0;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Records an internal inconsistency; the caller then skips the access that
// would have gone out of bounds and the run reports BFS_EDEVICE.
__device__ __forceinline__ void flag_internal(Ctrl* c) {
    __hip_atomic_store(&c->error, BFS_EINTERNAL_CODE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- look-back descriptors ---------------------------------------------------------------
// [63:62] status (0 empty, 1 tile aggregate, 2 inclusive prefix), [61:31] count, [30:0] edges.
__device__ __forceinline__ unsigned long long pack_desc(unsigned st, unsigned cnt, unsigned sum) {
    return ((unsigned long long)st << 62) | ((unsigned long long)(cnt & 0x7fffffffu) << 31) |
           (unsigned long long)(sum & 0x7fffffffu);
}
__device__ __forceinline__ unsigned desc_st(unsigned long long d) { return (unsigned)(d >> 62); }
__device__ __forceinline__ unsigned desc_cnt(unsigned long long d) { return (unsigned)(d >> 31) & 0x7fffffffu; }
__device__ __forceinline__ unsigned desc_sum(unsigned long long d) { return (unsigned)d & 0x7fffffffu; }

// Thread 0 publishes tile k's aggregate and looks back for its exclusive
// prefix.  Returns false on a failed wait.
__device__ bool lookback(unsigned long long* desc, int k, int agg_c, int agg_s, Ctrl* c, uint64_t spin_ticks,
                         int* pre_c, int* pre_s) {
    if (k == 0) {
        st_rel(&desc[0], pack_desc(2, agg_c, agg_s));
        *pre_c = 0;
        *pre_s = 0;
        return true;
    }
    st_rel(&desc[k], pack_desc(1, agg_c, agg_s));
    unsigned ac = 0, as = 0;
    int j = k - 1;
    for (;;) {
        unsigned long long d = ld_acq(&desc[j]);
        if (desc_st(d) == 0) {
            if (!spin_until(c, spin_ticks, [&] { return desc_st(d = ld_acq(&desc[j])) != 0; })) return false;
        }
        ac += desc_cnt(d);
        as += desc_sum(d);
        if (desc_st(d) == 2) break;
        --j;
    }
    st_rel(&desc[k], pack_desc(2, ac + agg_c, as + agg_s));
    *pre_c = (int)ac;
    *pre_s = (int)as;
    return true;
}

// Marks every share that starts inside [e, e + d) as starting at frontier entry pos.
__device__ __forceinline__ void scatter_starts(const Params& p, int32_t* tstart, int pos, int e, int d) {
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

// ---- compaction of one tile's private queue ----------------------------------------------
// l is the level whose candidates are compacted (-1 for the roots); the
// survivors form the frontier of level l + 1.
__device__ bool compact_tile(const Params& p, int l, int k, int ntiles, int* lds) {
    int* s_wave = lds + kLdsWords - 2 * kWaves - 8;
    int* s_wave2 = s_wave + kWaves;
    int* s_b = s_wave2 + kWaves;
    const int par = l & 1;
    const int np = (l + 1) & 1;
    int c = p.cnt[k];
    if (c < 0 || c > kGrain) {
        if (threadIdx.x == 0) flag_internal(p.ctrl);
        c = 0;
    }
    int v[kVT], rs[kVT], d[kVT];
    int tc = 0, ts = 0, traw = 0;
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        const int idx = i * kBlock + threadIdx.x;
        v[i] = -1;
        if (idx < c) {
            const int slot = k * kGrain + idx;
            const int vv = p.cand[slot];
            if ((unsigned)vv >= (unsigned)p.n) flag_internal(p.ctrl);
            else if (p.owner[vv] == slot) v[i] = vv;
        }
    }
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        d[i] = 0;
        rs[i] = 0;
        if (v[i] >= 0) {
            rs[i] = p.offsets[v[i]];
            d[i] = p.offsets[v[i] + 1] - rs[i];
            ++traw;
            if (d[i] > 0) { ++tc; ts += d[i]; }
        }
    }
    int C, S, R;
    const int c_ex = block_excl_scan(tc, s_wave, &C);
    const int s_ex = block_excl_scan(ts, s_wave2, &S);
    block_excl_scan(traw, s_wave, &R);  // survivors of any degree: only the total is used
    if (threadIdx.x == 0) {
        int pc = 0, ps = 0;
        bool ok = lookback(p.desc[par], k, C, S, p.ctrl, p.spin_ticks, &pc, &ps);
        s_b[0] = pc;
        s_b[1] = ps;
        s_b[2] = ok;
        if (R) __hip_atomic_fetch_add(&p.ctrl->kept[np], R, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ok && k == ntiles - 1) {
            st_rel(&p.ctrl->nl[np], pc + C);
            st_rel(&p.ctrl->el[np], ps + S);
            if (pc + C <= p.n) p.f_ex[np][pc + C] = ps + S;
            else flag_internal(p.ctrl);
        }
    }
    __syncthreads();
    const int pc = s_b[0], ps = s_b[1];
    const bool ok = s_b[2] != 0;
    __syncthreads();
    if (!ok) return false;
    int pos = pc + c_ex, e = ps + s_ex;
    int32_t* frs = p.f_rs[np];
    int32_t* fex = p.f_ex[np];
    int32_t* tst = p.tstart[np];
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        if (v[i] >= 0) {
            __hip_atomic_fetch_or(&p.bitmap[v[i] >> 5], 1u << (v[i] & 31), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            if (d[i] > 0) {
                if ((unsigned)pos < (unsigned)p.n) {
                    frs[pos] = rs[i];
                    fex[pos] = e;
                    scatter_starts(p, tst, pos, e, d[i]);
                } else {
                    flag_internal(p.ctrl);
                }
                ++pos;
                e += d[i];
            }
        }
    }
    return true;
}

// Ticket-ordered loop over the compaction tiles of level l.
__device__ bool compact_phase(const Params& p, int l, int ntiles, int* lds) {
    int* s_b = lds + kLdsWords - 8;
    const int par = l & 1;
    for (;;) {
        if (threadIdx.x == 0)
            s_b[4] = (int)__hip_atomic_fetch_add(&p.ctrl->ticket[par], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int k = s_b[4];
        __syncthreads();
        if (k >= ntiles) return true;
        if (!compact_tile(p, l, k, ntiles, lds)) return false;
    }
}

// ---- expansion of one share ---------------------------------------------------------------
__device__ void expand_tile(const Params& p, int l, int k, int ntiles, int n_l, int e_l, int* lds) {
    int* s_ex = lds;
    int* s_rs = lds + kGrain + 1;
    int* s_wave = lds + kLdsWords - 2 * kWaves - 8;
    const int par = l & 1;
    const int g0 = k * kGrain;
    const int g1 = min(g0 + kGrain, e_l);
    const int32_t* tst = p.tstart[par];
    const int j0 = tst[k];
    const int j1 = (k + 1 < ntiles) ? tst[k + 1] : n_l - 1;
    const int nv = j1 - j0 + 1;  // <= kGrain + 1: every frontier vertex has degree >= 1
    if (j0 < 0 || j1 >= n_l || nv < 1 || nv > kGrain + 1 || k >= p.max_tiles) {
        // cannot happen for a well-formed frontier; refuse rather than overrun LDS
        if (threadIdx.x == 0) {
            flag_internal(p.ctrl);
            p.cnt[k < p.max_tiles ? k : 0] = 0;
        }
        __syncthreads();
        return;
    }
    const int32_t* fex = p.f_ex[par];
    const int32_t* frs = p.f_rs[par];
    for (int i = threadIdx.x; i < nv; i += kBlock) {
        s_ex[i] = fex[j0 + i];
        s_rs[i] = frs[j0 + i];
    }
    __syncthreads();
    int v[kVT];
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        const int g = g0 + i * kBlock + threadIdx.x;
        v[i] = -1;
        if (g < g1) {
            int lo = 0, hi = nv;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_ex[mid] <= g) lo = mid; else hi = mid;
            }
            const int idx = s_rs[lo] + (g - s_ex[lo]);
            if ((unsigned)idx < (unsigned)p.m) {
                v[i] = __builtin_nontemporal_load(p.cols + idx);
                if ((unsigned)v[i] >= (unsigned)p.n) v[i] = -1;
            } else {
                flag_internal(p.ctrl);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kVT; ++i)
        if (v[i] >= 0 && ((p.bitmap[v[i] >> 5] >> (v[i] & 31)) & 1u)) v[i] = -1;
#pragma unroll
    for (int i = 0; i < kVT; ++i)
        if (v[i] >= 0 && p.level[v[i]] != -1) v[i] = -1;
#pragma unroll
    for (int i = 0; i < kVT; ++i)
        if (v[i] >= 0) p.level[v[i]] = l + 1;
    int slot[kVT];
    int wt = 0;
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        const uint64_t b = ballot(v[i] >= 0);
        slot[i] = wt + mbcnt(b);
        wt += __popcll(b);
    }
    if (lane_id() == 0) s_wave[wave_id()] = wt;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int t = s_wave[w];
        base += (w < wave_id()) ? t : 0;
        tot += t;
    }
#pragma unroll
    for (int i = 0; i < kVT; ++i) {
        if (v[i] >= 0) {
            const int s = k * kGrain + base + slot[i];
            p.owner[v[i]] = s;
            p.cand[s] = v[i];
        }
    }
    if (threadIdx.x == 0) p.cnt[k] = tot;
    __syncthreads();
}

// ---- a stretch of small levels run by one workgroup out of LDS -----------------------------
// Entered at level l with the frontier in global memory (parity l & 1).
// Leaves with the frontier of level ctrl->resume in global memory.
__device__ void small_levels(const Params& p, int l, int n_l, int e_l, int* lds) {
    int* s_rs = lds;
    int* s_ex = lds + kSmallN;
    int* s_cand = s_ex + kSmallN + 1;
    int* s_wave = lds + kLdsWords - 2 * kWaves - 8;
    int* s_wave2 = s_wave + kWaves;
    {
        const int par = l & 1;
        for (int i = threadIdx.x; i < n_l; i += kBlock) {
            s_rs[i] = p.f_rs[par][i];
            s_ex[i] = p.f_ex[par][i];
        }
        if (threadIdx.x == 0) s_ex[n_l] = e_l;
        __syncthreads();
    }
    int done_levels = 0;
    for (;;) {
        const int np = (l + 1) & 1;
        // expand level l: every frontier edge, kBlock * kVTS per round
        int ncand = 0;
        for (int base0 = 0; base0 < e_l; base0 += kBlock * kVTS) {
            int v[kVTS];
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                const int g = base0 + i * kBlock + threadIdx.x;
                v[i] = -1;
                if (g < e_l) {
                    int lo = 0, hi = n_l;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_ex[mid] <= g) lo = mid; else hi = mid;
                    }
                    const int idx = s_rs[lo] + (g - s_ex[lo]);
                    if ((unsigned)idx < (unsigned)p.m) {
                        v[i] = p.cols[idx];
                        if ((unsigned)v[i] >= (unsigned)p.n) v[i] = -1;
                    } else {
                        flag_internal(p.ctrl);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < kVTS; ++i)
                if (v[i] >= 0 && p.level[v[i]] != -1) v[i] = -1;
#pragma unroll
            for (int i = 0; i < kVTS; ++i)
                if (v[i] >= 0) p.level[v[i]] = l + 1;
            int slot[kVTS];
            int wt = 0;
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                const uint64_t b = ballot(v[i] >= 0);
                slot[i] = wt + mbcnt(b);
                wt += __popcll(b);
            }
            if (lane_id() == 0) s_wave[wave_id()] = wt;
            __syncthreads();
            int wb = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const int t = s_wave[w];
                wb += (w < wave_id()) ? t : 0;
                tot += t;
            }
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                if (v[i] >= 0) {
                    const int s = ncand + wb + slot[i];
                    p.owner[v[i]] = s;
                    if (s < kSmallC) s_cand[s] = v[i]; else p.cand[s] = v[i];
                }
            }
            ncand += tot;
            __syncthreads();
        }
        // de-duplicate and build the next frontier (LDS and global copies)
        int outc = 0, outs = 0, outr = 0;
        for (int base0 = 0; base0 < ncand; base0 += kBlock * kVTS) {
            int v[kVTS], rs[kVTS], d[kVTS];
            int tc = 0, ts = 0, tr = 0;
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                const int idx = base0 + i * kBlock + threadIdx.x;
                v[i] = -1;
                if (idx < ncand) {
                    const int vv = idx < kSmallC ? s_cand[idx] : p.cand[idx];
                    if ((unsigned)vv >= (unsigned)p.n) flag_internal(p.ctrl);
                    else if (p.owner[vv] == idx) v[i] = vv;
                }
            }
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                rs[i] = 0;
                d[i] = 0;
                if (v[i] >= 0) {
                    rs[i] = p.offsets[v[i]];
                    d[i] = p.offsets[v[i] + 1] - rs[i];
                    ++tr;
                    if (d[i] > 0) { ++tc; ts += d[i]; }
                }
            }
            int C, S, R;
            const int c_ex = block_excl_scan(tc, s_wave, &C);
            const int s_ex2 = block_excl_scan(ts, s_wave2, &S);
            block_excl_scan(tr, s_wave, &R);
            int pos = outc + c_ex, e = outs + s_ex2;
#pragma unroll
            for (int i = 0; i < kVTS; ++i) {
                if (v[i] >= 0) {
                    __hip_atomic_fetch_or(&p.bitmap[v[i] >> 5], 1u << (v[i] & 31), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                    if (d[i] > 0) {
                        if ((unsigned)pos < (unsigned)p.n) {
                            p.f_rs[np][pos] = rs[i];
                            p.f_ex[np][pos] = e;
                            scatter_starts(p, p.tstart[np], pos, e, d[i]);
                        } else {
                            flag_internal(p.ctrl);
                        }
                        if (pos < kSmallN) {
                            s_rs[pos] = rs[i];
                            s_ex[pos] = e;
                        }
                        ++pos;
                        e += d[i];
                    }
                }
            }
            outc += C;
            outs += S;
            outr += R;
            __syncthreads();
        }
        ++l;
        ++done_levels;
        if (threadIdx.x == 0) {
            if (outc <= p.n) p.f_ex[np][outc] = outs;
            if (outr > 0 && l < kStatCap) {
                p.stat_nl[l] = outr;
                p.stat_el[l] = outs;
            }
            if (outr > 0) st_rel(&p.ctrl->levels, l + 1);
            st_rel(&p.ctrl->heartbeat, l);
        }
        n_l = outc;
        e_l = outs;
        if (n_l == 0 || n_l > kSmallN || e_l > p.small_edges) {
            // hand the frontier back through the resume slot: the parity slots
            // may still be read by workgroups that have not left the level the
            // stretch started at
            if (threadIdx.x == 0) {
                st_rel(&p.ctrl->r_nl, n_l);
                st_rel(&p.ctrl->r_el, e_l);
                st_rel(&p.ctrl->r_kept, outr);
                st_rel(&p.ctrl->resume, l);
                __hip_atomic_fetch_add(&p.ctrl->small_levels, done_levels, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            return;
        }
        if (threadIdx.x == 0) s_ex[n_l] = e_l;
        __syncthreads();
    }
}

// ---- parent pass ------------------------------------------------------------------------------
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

// Resets the control block and the per-run arrays: level = -1, bitmap = 0,
// and the descriptors of the roots' compaction.
__global__ void __launch_bounds__(kBlock) k_prep(Params p, int prep_tiles) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = tid; v < p.n; v += stride) p.level[v] = -1;
    const int64_t words = ((int64_t)p.n + 31) >> 5;
    for (int64_t w = tid; w < words; w += stride) p.bitmap[w] = 0u;
    for (int64_t t = tid; t < prep_tiles; t += stride) p.desc[1][t] = 0ull;
    if (tid == 0) {
        Ctrl* c = p.ctrl;
        c->bar = 0;
        c->ticket[0] = c->ticket[1] = 0;
        c->nl[0] = c->nl[1] = 0;
        c->el[0] = c->el[1] = 0;
        c->kept[0] = c->kept[1] = 0;
        c->levels = 0;
        c->error = 0;
        c->small_levels = 0;
        c->resume = 0;
        c->heartbeat = 0;
        c->plain_next = 0;
    }
}

// Roots become the private queues of level -1: root i sits in slot i.
__device__ void roots_range(const Params& p, int64_t first, int64_t stride) {
    for (int64_t i = first; i < p.nroots; i += stride) {
        const int r = p.roots ? p.roots[i] : p.single_root;
        p.level[r] = 0;
        p.owner[r] = (int)i;
        p.cand[i] = r;
        if ((i % kGrain) == 0) p.cnt[i / kGrain] = (int)min((int64_t)kGrain, (int64_t)p.nroots - i);
    }
}

__global__ void __launch_bounds__(kBlock) k_persistent(Params p) {
    __shared__ Lds lds_s;
    int* lds = lds_s.w;
    int* s_flag = lds + kLdsWords - 1;
    const int G = gridDim.x;
    Ctrl* c = p.ctrl;

    roots_range(p, (int64_t)blockIdx.x * kBlock + threadIdx.x, (int64_t)G * kBlock);
    if (!grid_barrier(c, p.spin_ticks, s_flag)) return;
    const int root_tiles = (p.nroots + kGrain - 1) / kGrain;
    if (!compact_phase(p, -1, root_tiles, lds)) return;
    if (!grid_barrier(c, p.spin_ticks, s_flag)) return;

    // The size of each level is read once, right after the barrier that
    // publishes it, into loop-carried values: the slot it came from may be
    // rewritten before every workgroup would otherwise have read it again.
    int l = 0;
    int n_l = ld_acq(&c->nl[0]);
    int e_l = ld_acq(&c->el[0]);
    int kept = ld_acq(&c->kept[0]);
    for (;;) {
        const int par = l & 1;
        if (blockIdx.x == 0 && threadIdx.x == 0 && kept > 0) {
            if (l < kStatCap) { p.stat_nl[l] = kept; p.stat_el[l] = e_l; }
            st_rel(&c->levels, l + 1);
        }
        if (n_l == 0) break;
        if (p.small_edges > 0 && n_l <= kSmallN && e_l <= p.small_edges) {
            if (blockIdx.x == 0) small_levels(p, l, n_l, e_l, lds);
            if (!grid_barrier(c, p.spin_ticks, s_flag)) return;
            l = ld_acq(&c->resume);
            n_l = ld_acq(&c->r_nl);
            e_l = ld_acq(&c->r_el);
            kept = ld_acq(&c->r_kept);
            continue;
        }
        const int ntiles = (int)(((int64_t)e_l + kGrain - 1) / kGrain);
        const int np = (l + 1) & 1;
        // reset this level's compaction state (last used two levels ago)
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st_rel(&c->ticket[par], 0u);
            st_rel(&c->kept[np], 0);
        }
        for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < ntiles; t += (int64_t)G * kBlock)
            p.desc[par][t] = 0ull;
        for (int k = blockIdx.x; k < ntiles; k += G) expand_tile(p, l, k, ntiles, n_l, e_l, lds);
        if (!grid_barrier(c, p.spin_ticks, s_flag)) return;
        if (!compact_phase(p, l, ntiles, lds)) return;
        if (!grid_barrier(c, p.spin_ticks, s_flag)) return;
        ++l;
        n_l = ld_acq(&c->nl[np]);
        e_l = ld_acq(&c->el[np]);
        kept = ld_acq(&c->kept[np]);
    }
    if (p.parent) parent_range(p, (int64_t)blockIdx.x * kBlock + threadIdx.x, (int64_t)G * kBlock);
}

// ---- per-level launches (BFS_MODE_LEVEL) ---------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_level_roots(Params p) {
    roots_range(p, (int64_t)blockIdx.x * kBlock + threadIdx.x, (int64_t)gridDim.x * kBlock);
}

__global__ void __launch_bounds__(kBlock) k_level_compact(Params p, int l, int ntiles) {
    __shared__ Lds lds_s;
    compact_phase(p, l, ntiles, lds_s.w);
}

__global__ void __launch_bounds__(kBlock) k_level_expand(Params p, int l, int ntiles) {
    __shared__ Lds lds_s;
    const int n_l = ld_acq(&p.ctrl->nl[l & 1]);
    const int e_l = ld_acq(&p.ctrl->el[l & 1]);
    const int par = l & 1, np = (l + 1) & 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st_rel(&p.ctrl->ticket[par], 0u);
        st_rel(&p.ctrl->kept[np], 0);
    }
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * kBlock)
        p.desc[par][t] = 0ull;
    for (int k = blockIdx.x; k < ntiles; k += gridDim.x) expand_tile(p, l, k, ntiles, n_l, e_l, lds_s.w);
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

// ---- primitive test kernel ---------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_prim_compact(Params p, int ntiles, int32_t* totals) {
    __shared__ Lds lds_s;
    compact_phase(p, 0, ntiles, lds_s.w);
    __syncthreads();
    (void)totals;
}

__global__ void k_prim_reset(Params p, int ntiles) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t t = tid; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) p.desc[0][t] = 0ull;
    if (tid == 0) {
        p.ctrl->ticket[0] = 0;
        p.ctrl->kept[1] = 0;
        p.ctrl->nl[1] = 0;
        p.ctrl->el[1] = 0;
        p.ctrl->error = 0;
    }
}

__global__ void k_prim_totals(Params p, int32_t* totals) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        totals[0] = p.ctrl->nl[1];
        totals[1] = p.ctrl->el[1];
    }
}

// ---- host launchers ----------------------------------------------------------------------------

int persistent_grid_capacity(int device) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_persistent),
                                                     kBlock, 0) != hipSuccess)
        return 0;
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

hipError_t launch_prep(const Params& p, int prep_tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_prep, dim3(fill_grid(p.n)), dim3(kBlock), 0, s, p, prep_tiles);
    return hipGetLastError();
}

hipError_t launch_persistent(const Params& p, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_persistent, dim3(grid), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_level_roots(const Params& p, hipStream_t s) {
    hipLaunchKernelGGL(k_level_roots, dim3(fill_grid(p.nroots)), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_level_compact(const Params& p, int l, int ntiles, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_level_compact, dim3(grid), dim3(kBlock), 0, s, p, l, ntiles);
    return hipGetLastError();
}

hipError_t launch_level_expand(const Params& p, int l, int ntiles, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_level_expand, dim3(grid), dim3(kBlock), 0, s, p, l, ntiles);
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
                               const int32_t* cnt, int32_t ntiles, int32_t* out_rs, int32_t* out_ex,
                               int32_t* out_tstart, int32_t tstart_cap, int32_t* totals, unsigned long long* desc,
                               Ctrl* ctrl, uint32_t* bitmap, hipStream_t s) {
    Params p{};
    p.offsets = offsets;
    p.n = n;
    p.max_tiles = tstart_cap;
    p.owner = const_cast<int32_t*>(owner);
    p.cand = const_cast<int32_t*>(cand);
    p.cnt = const_cast<int32_t*>(cnt);
    p.f_rs[1] = out_rs;
    p.f_ex[1] = out_ex;
    p.tstart[1] = out_tstart;
    p.desc[0] = desc;
    p.ctrl = ctrl;
    p.bitmap = bitmap;
    p.spin_ticks = 300000000ull;
    hipLaunchKernelGGL(k_prim_reset, dim3(fill_grid(ntiles)), dim3(kBlock), 0, s, p, ntiles);
    int g = ntiles < 1024 ? (ntiles > 0 ? ntiles : 1) : 1024;
    hipLaunchKernelGGL(k_prim_compact, dim3(g), dim3(kBlock), 0, s, p, ntiles, totals);
    hipLaunchKernelGGL(k_prim_totals, dim3(1), dim3(64), 0, s, p, totals);
    return hipGetLastError();
}

}  // namespace s3bfs
