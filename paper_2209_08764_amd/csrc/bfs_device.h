// Device-side building blocks shared by the single-source and batched level
// loops: wave/workgroup scans, ballots, bounded waits, the grid barrier and
// the decoupled look-back over 64-bit (count, edge sum) descriptors.
#pragma once

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

// Workgroup barrier that orders LDS only.  A full __syncthreads() also
// waits for every outstanding global load, store and atomic of the wave;
// this one lets them stay in flight (prefetched loads, fire-and-forget
// stores), so it may only be used where no lane reads global data another
// lane of the workgroup wrote since the last full barrier.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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

// For each of N edge indices g[i], the entry lo[i] of a sorted array of
// exclusive degree sums ex[0..nv) with ex[lo] <= g[i] < ex[lo + 1] (the
// frontier entry owning the edge).  The N searches advance in lockstep, so
// their LDS reads are in flight together instead of one search after another.
// ex[0] <= g[i] is assumed; every search takes ceil(log2 nv) steps.
template <int N>
__device__ __forceinline__ void search_owners(const int* ex, int nv, const int* g, int* lo) {
    int hi[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        lo[i] = 0;
        hi[i] = nv;
    }
    const int steps = nv > 1 ? 32 - __builtin_clz((unsigned)(nv - 1)) : 0;
    for (int s = 0; s < steps; ++s) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int mid = (lo[i] + hi[i]) >> 1;   // mid == lo once the range holds one entry
            const bool right = ex[mid] <= g[i];
            lo[i] = right ? mid : lo[i];
            hi[i] = right ? hi[i] : mid;
        }
    }
}

// Exclusive block-wide prefix sum of one int per thread; *total gets the sum.
// s_tmp holds kWaves ints.  Must be called by the whole workgroup; orders
// LDS only.
__device__ __forceinline__ int block_excl_scan(int x, int* s_tmp, int* total) {
    const int incl = wave_incl_scan(x);
    if (lane_id() == 63) s_tmp[wave_id()] = incl;
    lds_barrier();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int t = s_tmp[w];
        base += (w < wave_id()) ? t : 0;
        tot += t;
    }
    lds_barrier();
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
__device__ inline bool spin_until(Ctrl* c, uint64_t spin_ticks, Pred pred) {
    uint64_t t0 = now_ticks();
    int hb = ld_acq(&c->heartbeat);
    // the condition is polled every time, the error and heartbeat words every 32nd time: a
    // waiting workgroup adds little traffic next to the ones still at work
    for (int polls = 1; !pred(); ++polls) {
        __builtin_amdgcn_s_sleep(1);
        if (polls & 31) continue;
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
__device__ inline bool grid_barrier(Ctrl* c, uint64_t spin_ticks, int* s_flag) {
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

// Hardware id of the XCD the wave runs on (the XCC_ID register, id 20).
__device__ __forceinline__ int xcd_id() {
    return (int)(__builtin_amdgcn_s_getreg((31 << 11) | 20) & (unsigned)(kMaxXcd - 1));
}

// A workgroup's place in the XCD-grouped barrier; only thread 0 holds it.
struct XGroup {
    int xcd;                  // the workgroup's XCD
    int groups;               // XCDs that hold workgroups of the launch
    unsigned long long size;  // workgroups of the launch on this XCD
};

// Thread 0 registers its workgroup on its XCD before a grid_barrier and
// reads the group sizes with xbar_group after it.
__device__ __forceinline__ void xbar_join(XBar* xb, int xcd) {
    __hip_atomic_fetch_add(&xb->wgs[xcd * kXLine], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline XGroup xbar_group(const XBar* xb, int xcd) {
    XGroup g{xcd, 0, ld_acq(&xb->wgs[xcd * kXLine])};
    for (int x = 0; x < kMaxXcd; ++x) g.groups += ld_acq(&xb->wgs[x * kXLine]) != 0ull;
    return g;
}

// Grid barrier grouped by XCD, for the same resident grids as grid_barrier.
// An agent-scope release writes back the whole L2 of the XCD that issues it,
// whichever CU wrote the dirty lines, and the XCD's workgroups issuing one
// each in turn made the flat barrier cost about 20 us at 512 workgroups.
// Here every wave first waits until the L2 has acknowledged its own stores
// and atomics; the last workgroup of an XCD to arrive then writes that L2
// back once for all of them and arrives at the top counter.  The last XCD
// there releases the per-XCD copies of the generation, which each workgroup
// polls on its own XCD's line before invalidating its caches.
__device__ inline bool xcd_barrier(Ctrl* c, XBar* xb, const XGroup& g, uint64_t spin_ticks, int* s_flag) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's accesses have been acknowledged
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long a =
            __hip_atomic_fetch_add(&xb->arrive[g.xcd * kXLine], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long gen = a / g.size + 1;
        if (a % g.size == g.size - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");  // the XCD's L2 write-back
            const unsigned long long t =
                __hip_atomic_fetch_add(&xb->top[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t % (unsigned)g.groups == (unsigned)g.groups - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                for (int x = 0; x < kMaxXcd; ++x) st_rel(&xb->gen[x * kXLine], gen);
            }
        }
        const bool ok = spin_until(c, spin_ticks, [&] { return ld_acq(&xb->gen[g.xcd * kXLine]) >= gen; });
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_flag = ok && ld_acq(&c->error) == 0;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Barrier of a lite level's P active workgroups (the first P).  Each active
// workgroup arrives after an agent-scope release; the last one resets the
// counter for the next such barrier and publishes `gen` on every XCD's line.
// Workgroups that do not take part (participate = false) only wait for the
// generation, which hands them the level's results; generations grow within a
// launch.  Grid barriers count every workgroup of the launch, so a lite level
// uses this one for both of its barriers, and no workgroup arrives at a grid
// barrier meanwhile.
//
// release = false: the workgroup wrote nothing since the last barrier that others read with plain
// loads (only atomics, which are coherent on every XCD), so it skips the write-back of its XCD's
// L2 and only waits until its own atomics have been performed before arriving.
__device__ inline bool sub_barrier(Ctrl* c, XBar* xb, int xcd, unsigned long long gen, int P, bool participate,
                                   uint64_t spin_ticks, int* s_flag, bool release = true) {
    if (!release) __builtin_amdgcn_s_waitcnt(0);  // this wave's atomics have been performed
    __syncthreads();
    if (threadIdx.x == 0) {
        if (participate) {
            if (release) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned long long a =
                __hip_atomic_fetch_add(&xb->pcnt[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a == (unsigned long long)P - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                st_rel(&xb->pcnt[0], 0ull);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                for (int x = 0; x < kMaxXcd; ++x) st_rel(&xb->pgen[x * kXLine], gen);
            }
        }
        const bool ok = spin_until(c, spin_ticks, [&] { return ld_acq(&xb->pgen[xcd * kXLine]) >= gen; });
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

// Wave 0 publishes tile k's aggregate and looks back for its exclusive
// prefix, 64 predecessors per step: every lane loads one descriptor, the
// closest inclusive prefix is found with a ballot, and the aggregates in
// between are summed across the wave.  Must be called by all 64 lanes of one
// wave.  Returns false on a failed wait.
__device__ inline bool lookback_wave(unsigned long long* desc, int k, int agg_c, int agg_s, Ctrl* c,
                              uint64_t spin_ticks, int* pre_c, int* pre_s) {
    const int lane = lane_id();
    if (k == 0) {
        if (lane == 0) st_rel(&desc[0], pack_desc(2, agg_c, agg_s));
        *pre_c = 0;
        *pre_s = 0;
        return true;
    }
    if (lane == 0) st_rel(&desc[k], pack_desc(1, agg_c, agg_s));
    int acc_c = 0, acc_s = 0;
    int base = k - 1;
    uint64_t t0 = now_ticks();
    for (;;) {
        const int j = base - lane;
        const unsigned long long d = j >= 0 ? ld_acq(&desc[j]) : pack_desc(2, 0, 0);
        const unsigned st = desc_st(d);
        const uint64_t b0 = ballot(st == 0);
        const uint64_t b2 = ballot(st == 2);
        // lanes up to and including the closest inclusive prefix (or all 64)
        const int last = b2 ? __builtin_ctzll(b2) : 63;
        const uint64_t need = last == 63 ? ~0ull : ((1ull << (last + 1)) - 1);
        if (b0 & need) {
            // a closer predecessor has not published yet: wait and reload
            __builtin_amdgcn_s_sleep(1);
            if (now_ticks() - t0 > spin_ticks || ld_acq(&c->error) != 0) {
                if (lane == 0)
                    __hip_atomic_store(&c->error, BFS_EDEVICE_CODE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            continue;
        }
        const bool take = lane <= last;
        const int vc = take ? (int)desc_cnt(d) : 0;
        const int vs = take ? (int)desc_sum(d) : 0;
        acc_c += __builtin_amdgcn_readlane(wave_incl_scan(vc), 63);
        acc_s += __builtin_amdgcn_readlane(wave_incl_scan(vs), 63);
        if (b2) break;
        base -= 64;
        t0 = now_ticks();
    }
    if (lane == 0) st_rel(&desc[k], pack_desc(2, acc_c + agg_c, acc_s + agg_s));
    *pre_c = acc_c;
    *pre_s = acc_s;
    return true;
}


}  // namespace s3bfs
