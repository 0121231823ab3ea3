// Batched multi-source search: k <= 256 searches in one level loop, each
// vertex carrying 4 x 64-bit masks (bit j = source j): frontier F, next N
// and visited V.  Per level l:
//
//   expand  push (few active edges): every edge (u, v) of an active vertex u
//           ORs F[u] into N[v] with 64-bit atomics, load-balanced over the
//           active list with the same share / sub-tile split as the
//           single-source loop (the paper's equal division of e_l);
//           pull (many active edges): every vertex of degree >= 1 that still
//           misses some source ORs F[u] over its active neighbours u (active
//           bitmap in L2) into an LDS accumulator; only rows cut by a
//           sub-tile boundary go to N[v] atomically.
//   update  a dense pass over the vertices: new = N & ~V, V |= new, F = new,
//           level byte l + 1 for every new bit (byte-masked wave stores of
//           the vertex's row), N = 0, and the next active list with its
//           degree prefix sums and sub-tile start points by decoupled
//           look-back over update tiles (the Sizes prefix sum again).
//   next    one lane advances the level and stops the loop when no vertex is
//           active or a level would not fit in a byte.
//   hotmask before a pull level on a graph with hot-vertex numbering: the
//           hot vertices' masks copied into a compact array indexed by hot
//           number, which the pull gathers from instead of F.
//
// OR is commutative and idempotent, so the result does not depend on the
// order of the atomics or on push versus pull.  The level loop is replayed
// from a captured hipGraph; every kernel returns at once after the stop.  A
// one-workgroup kernel behind the replays runs whatever levels they left, so
// the host never waits between replays.
#include "bfs_device.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace s3bfs {

namespace {

__device__ __forceinline__ void bshare_range(int b, int P, int ntiles, int* tb, int* te) {
    *tb = (int)(((int64_t)b * ntiles) / P);
    *te = (int)(((int64_t)(b + 1) * ntiles) / P);
}

__device__ __forceinline__ void bflag(Ctrl* c) {
    __hip_atomic_store(&c->error, BFS_EINTERNAL_CODE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sub-tile start points: entry pos (edges [e, e + d)) starts every sub-tile
// of G = kBlock * BVT edges that begins inside its edge range.
template <int BVT>
__device__ __forceinline__ void bscatter(const BatchParams& p, int32_t* ts, int pos, int64_t e, int d) {
    constexpr int G = kBlock * BVT;
    int64_t t = (e + G - 1) / G;
    const int64_t tend = (e + d + G - 1) / G;
    if (t < 0 || tend > p.max_tiles) {
        bflag(p.ctrl);
        return;
    }
    for (; t < tend; ++t) ts[t] = pos;
}

// A vertex's four 64-bit mask words (32-byte aligned), read as two 16-byte loads whatever the
// batch's word count: the loads then carry no branches, each of which would make the next load
// wait for the one before it.  Words past the batch's count may hold an earlier batch's bits and
// are never used.
struct alignas(16) Mask2 {
    unsigned long long a, b;
};
__device__ __forceinline__ void load_mask(const unsigned long long* src, unsigned long long* f) {
    const Mask2* q = reinterpret_cast<const Mask2*>(src);
    const Mask2 lo = q[0], hi = q[1];
    f[0] = lo.a;
    f[1] = lo.b;
    f[2] = hi.a;
    f[3] = hi.b;
}

template <int BVT>
struct ExpLds {
    static constexpr int kSl = kBlock * BVT + 1;   // slice entries of one sub-tile
    unsigned long long acc[kSl * 4];               // pull accumulators (8 B aligned first)
    int sl[3 * kSl];                               // sub-tile slice: ex | rs | v
};

template <int UV>
struct UpdLds {
    int misc[2 * kWaves + 16 + kBlock * UV / 32];  // scan partials, look-back result, active bits
};

}  // namespace

// ---- one-off set-up: the vertices of degree >= 1 and the sub-tiles over all edges ----------
// nz_v lists them in ascending order; since isolated vertices own no edge,
// the edges before nz_v[j] are exactly offsets[nz_v[j]].
template <int BVT>
__global__ void __launch_bounds__(kBlock) k_batch_nz(BatchParams p) {
    constexpr int NV = kNzTile / kBlock;
    __shared__ UpdLds<NV> lds;
    int* s_wave = lds.misc;
    const int tile = blockIdx.x;
    const int v0 = tile * kNzTile + threadIdx.x * NV;
    int keep[NV], tc = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int v = v0 + i;
        keep[i] = v < p.n && p.offsets[v + 1] > p.offsets[v];
        tc += keep[i];
    }
    int C;
    const int pre = block_excl_scan(tc, s_wave, &C);
    int* s_b = lds.misc + 2 * kWaves;
    if (wave_id() == 0) {
        int pc = 0, ps = 0;
        const bool ok = lookback_wave(p.desc[0], tile, C, 0, p.ctrl, p.spin_ticks, &pc, &ps);
        if (threadIdx.x == 0) {
            s_b[0] = pc;
            s_b[1] = ok;
            if (ok && tile == (int)gridDim.x - 1) st_rel(&p.ctrl->nz_count, pc + C);
        }
    }
    lds_barrier();
    if (!s_b[1]) return;
    int pos = s_b[0] + pre;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (keep[i]) {
            const int v = v0 + i;
            p.nz_v[pos] = v;
            bscatter<BVT>(p, p.nz_ts, pos, p.offsets[v], p.offsets[v + 1] - p.offsets[v]);
            ++pos;
        }
    }
}

// ---- per run ---------------------------------------------------------------------------------

// level bytes = 255, V = N = 0, active bitmap = 0, control block reset.
__global__ void __launch_bounds__(kBlock) k_batch_prep(BatchParams p) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint8_t* level = p.args->level;
    const int64_t nbytes = level ? (int64_t)p.n * p.args->k : 0;
    uint32_t* l32 = reinterpret_cast<uint32_t*>(level);  // the caller's array is 4-byte aligned
    for (int64_t i = tid; i < nbytes / 4; i += stride) l32[i] = 0xffffffffu;
    for (int64_t i = (nbytes / 4) * 4 + tid; i < nbytes; i += stride) level[i] = 255;
    for (int64_t i = tid; i < (int64_t)p.n * 4; i += stride) {
        p.vis[i] = 0ull;
        p.nx[i] = 0ull;
    }
    for (int64_t i = tid; i < ((int64_t)p.n + 31) / 32; i += stride) p.act_bits[i] = 0u;
    for (int64_t i = tid; i < p.desc_cap; i += stride) p.desc[0][i] = 0ull;
    if (tid == 0) {
        Ctrl* c = p.ctrl;
        c->b_nact[0] = c->b_nact[1] = 0;
        c->b_eact[0] = c->b_eact[1] = 0;
        c->blevel = -1;
        c->bdone = 0;
        c->batch_overflow = 0;
        c->error = 0;
        c->levels = 0;
    }
}

// Bit j of N[sources[j]]: the sources become the "next" set of level -1.
__global__ void k_batch_seed(BatchParams p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int j = 0; j < p.args->k; ++j) {
            const int s = p.sources[j];
            p.nx[(int64_t)s * 4 + (j >> 6)] |= 1ull << (j & 63);
        }
    }
}

// Dense update after the expansion of level l (l = -1: the seeds): update tile `tile` of
// `ntiles` (the tiles' look-back chains them in index order).
template <int BVT, int UV>
__device__ __forceinline__ void batch_update_tile(const BatchParams& p, int tile, int ntiles, UpdLds<UV>& lds) {
    constexpr int UT = kBlock * UV;
    Ctrl* c = p.ctrl;
    if (ld_acq(&c->bdone)) return;
    const int l = ld_acq(&c->blevel);
    const int np = (l + 1) & 1;
    int* s_wave = lds.misc;
    int* s_wave2 = lds.misc + kWaves;
    int* s_b = lds.misc + 2 * kWaves;
    uint32_t* s_bits = reinterpret_cast<uint32_t*>(lds.misc + 2 * kWaves + 16);
    const int v0 = tile * UT + threadIdx.x * UV;
    const int W = p.args->words;
    const int K = p.args->k;
    uint8_t* level = p.args->level;
    const uint8_t lv = (uint8_t)(l + 1);
    const bool fits = l + 1 < 255;
    if (threadIdx.x < UT / 32) s_bits[threadIdx.x] = 0u;
    lds_barrier();
    int tc = 0, ts = 0;
    int act[UV], deg[UV], rs[UV];
    unsigned long long nw[UV][4];
    // this thread's UV vertices in phases, each phase's loads together: next-level masks,
    // then the visited masks of those reached, then the row offsets of the new ones
    unsigned long long nn[UV][4], vw[UV][4];
    bool any[UV];
#pragma unroll
    for (int i = 0; i < UV; ++i) {
        const int v = v0 + i;
        load_mask(p.nx + (int64_t)(v < p.n ? v : 0) * 4, nn[i]);
        any[i] = false;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if (w >= W || v >= p.n) nn[i][w] = 0ull;
            any[i] |= nn[i][w] != 0ull;
        }
    }
#pragma unroll
    for (int i = 0; i < UV; ++i) {
        if (any[i]) load_mask(p.vis + (int64_t)(v0 + i) * 4, vw[i]);
        else vw[i][0] = vw[i][1] = vw[i][2] = vw[i][3] = 0ull;
    }
    bool fresh[UV];
#pragma unroll
    for (int i = 0; i < UV; ++i) {
        const int v = v0 + i;
        act[i] = 0;
        deg[i] = 0;
        rs[i] = 0;
        fresh[i] = false;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            nw[i][w] = nn[i][w] & ~vw[i][w];
            fresh[i] |= nw[i][w] != 0ull;
        }
        if (any[i]) {
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if (w < W) {
                    p.nx[(int64_t)v * 4 + w] = 0ull;
                    if (nw[i][w]) p.vis[(int64_t)v * 4 + w] = vw[i][w] | nw[i][w];
                    p.fr[(int64_t)v * 4 + w] = nw[i][w];
                }
            }
        }
    }
    int o0[UV], o1[UV];
#pragma unroll
    for (int i = 0; i < UV; ++i) {
        if (fresh[i] && fits) {
            o0[i] = p.offsets[v0 + i];
            o1[i] = p.offsets[v0 + i + 1];
        }
    }
#pragma unroll
    for (int i = 0; i < UV; ++i) {
        if (fresh[i]) {
            if (!fits) {
                __hip_atomic_store(&c->batch_overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                act[i] = 1;
                rs[i] = o0[i];
                deg[i] = o1[i] - o0[i];
                atomicOr(&s_bits[(threadIdx.x * UV + i) >> 5], 1u << ((threadIdx.x * UV + i) & 31));
                if (deg[i] > 0) {
                    ++tc;
                    ts += deg[i];
                }
            }
        }
    }
    // level bytes: the wave writes each new vertex's row, lane q covering sources 4q..4q+3
#pragma unroll
    for (int i = 0; i < UV; ++i) {
        uint64_t todo = ballot(act[i] != 0);
        while (todo) {
            const int src_lane = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int v = __builtin_amdgcn_readfirstlane(__shfl(v0 + i, src_lane));
            unsigned long long m4[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) m4[w] = __shfl(nw[i][w], src_lane);
            const int q = lane_id();
            uint8_t* row = level + (int64_t)v * K;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = 4 * q + b;
                if (j < K && ((m4[j >> 6] >> (j & 63)) & 1ull)) row[j] = lv;
            }
        }
    }
    int C, S;
    const int pre_c = block_excl_scan(tc, s_wave, &C);
    const int pre_s = block_excl_scan(ts, s_wave2, &S);
    if (wave_id() == 0) {
        int pc = 0, ps = 0;
        const bool ok = lookback_wave(p.desc[np], tile, C, S, c, p.spin_ticks, &pc, &ps);
        if (threadIdx.x == 0) {
            s_b[0] = pc;
            s_b[1] = ps;
            s_b[2] = ok;
            if (ok && tile == ntiles - 1) {
                st_rel(&c->b_nact[np], pc + C);
                st_rel(&c->b_eact[np], ps + S);
                p.act_ex[np][pc + C] = ps + S;
            }
        }
    }
    lds_barrier();
    // active bitmap of the next level (the tile's vertices are UT / 32 whole words)
    if (threadIdx.x < UT / 32) {
        const int64_t wi = ((int64_t)tile * UT) / 32 + threadIdx.x;
        if (wi < ((int64_t)p.n + 31) / 32) p.act_bits[wi] = s_bits[threadIdx.x];
    }
    if (!s_b[2]) return;
    int pos = s_b[0] + pre_c;
    int64_t e = (int64_t)s_b[1] + pre_s;
#pragma unroll
    for (int i = 0; i < UV; ++i) {
        if (act[i] && deg[i] > 0) {
            if ((unsigned)pos < (unsigned)p.n) {
                p.act[np][pos] = v0 + i;
                p.act_rs[np][pos] = rs[i];
                p.act_ex[np][pos] = (int)e;
                bscatter<BVT>(p, p.act_ts[np], pos, e, deg[i]);
            } else {
                bflag(c);
            }
            ++pos;
            e += deg[i];
        }
    }
}

template <int BVT, int UV>
__global__ void __launch_bounds__(kBlock) k_batch_update(BatchParams p) {
    __shared__ UpdLds<UV> lds;
    batch_update_tile<BVT, UV>(p, blockIdx.x, gridDim.x, lds);
}

// Expansion of level l: push over the active edges or pull over all rows, as workgroup b of
// nb.
template <int BVT>
__device__ __forceinline__ void batch_expand(const BatchParams& p, int b, int nb, ExpLds<BVT>& lds) {
    constexpr int G = kBlock * BVT;
    constexpr int SL = ExpLds<BVT>::kSl;
    Ctrl* c = p.ctrl;
    if (ld_acq(&c->bdone)) return;
    const int l = ld_acq(&c->blevel);
    const int par = l & 1;
    const int n_a = ld_acq(&c->b_nact[par]);
    const int e_a = ld_acq(&c->b_eact[par]);
    const int W = p.args->words;
    const int K = p.args->k;
    // descriptors of this level's update (last used two levels ago)
    for (int64_t t = (int64_t)b * kBlock + threadIdx.x; t < p.utiles; t += (int64_t)nb * kBlock)
        p.desc[(l + 1) & 1][t] = 0ull;
    int* sl = lds.sl;
    if (e_a <= p.args->pull_edges) {
        // ---- push over the active list ----
        const int ntiles = (int)(((int64_t)e_a + G - 1) / G);
        const int P = ntiles < nb ? ntiles : nb;
        if (b >= P) return;
        int tb, te;
        bshare_range(b, P, ntiles, &tb, &te);
        const int32_t* ts = p.act_ts[par];
        for (int t = tb; t < te; ++t) {
            const int j0 = ts[t];
            const int j1 = t + 1 < ntiles ? ts[t + 1] : n_a - 1;
            const int nv = j1 - j0 + 1;
            if (j0 < 0 || j1 >= n_a || nv < 1 || nv > SL) {
                if (threadIdx.x == 0) bflag(c);
                return;
            }
            lds_barrier();
            for (int i = threadIdx.x; i < nv; i += kBlock) {
                sl[i] = p.act_ex[par][j0 + i];
                sl[SL + i] = p.act_rs[par][j0 + i];
                sl[2 * SL + i] = p.act[par][j0 + i];
            }
            lds_barrier();
            const int g0 = t * G, g1 = min(g0 + G, e_a);
            int gg[BVT], own[BVT];
#pragma unroll
            for (int r = 0; r < BVT; ++r) gg[r] = min(g0 + r * kBlock + (int)threadIdx.x, g1 - 1);
            search_owners<BVT>(sl, nv, gg, own);
            // every edge's target and source masks are read before any atomic goes out
            int tv[BVT];
            bool okr[BVT];
            unsigned long long f[BVT][4];
#pragma unroll
            for (int r = 0; r < BVT; ++r) {  // from a clamped position, checked afterwards
                const int g = g0 + r * kBlock + threadIdx.x;
                const int lo = own[r];
                const int idx = sl[SL + lo] + (g - sl[lo]);
                okr[r] = (unsigned)idx < (unsigned)p.m;
                tv[r] = p.cols[okr[r] ? idx : 0];
                if (g >= g1) okr[r] = true, tv[r] = -1;  // no edge: nothing to flag
            }
#pragma unroll
            for (int r = 0; r < BVT; ++r)
                if (!okr[r]) {
                    bflag(c);
                    tv[r] = -1;
                }
#pragma unroll
            for (int r = 0; r < BVT; ++r) {
                const int u = sl[2 * SL + own[r]];
                const bool ok = (unsigned)tv[r] < (unsigned)p.n;
                if (ok) load_mask(p.fr + (int64_t)u * 4, f[r]);
                else f[r][0] = f[r][1] = f[r][2] = f[r][3] = 0ull;
            }
#pragma unroll
            for (int r = 0; r < BVT; ++r) {
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    if (w < W && f[r][w]) atomicOr(&p.nx[(int64_t)tv[r] * 4 + w], f[r][w]);
            }
        }
        return;
    }
    // ---- pull over every row that still misses a source ----
    // A hot neighbour's masks come from the compact copy of the hot vertices' masks (a few MiB
    // that the L2 mostly holds), zero when it is not active; the others from F, behind the
    // active bitmap.
    const int nz = ld_acq(&c->nz_count);
    const int ntiles = (int)((p.m + G - 1) / G);
    const int P = ntiles < nb ? ntiles : nb;
    if (b >= P) return;
    int tb, te;
    bshare_range(b, P, ntiles, &tb, &te);
    unsigned long long full[4];
#pragma unroll
    for (int w = 0; w < 4; ++w)
        full[w] = w < W ? ((w + 1) * 64 <= K ? ~0ull : ((1ull << (K - w * 64)) - 1ull)) : 0ull;
    for (int t = tb; t < te; ++t) {
        const int j0 = p.nz_ts[t];
        const int j1 = t + 1 < ntiles ? p.nz_ts[t + 1] : nz - 1;
        const int nv = j1 - j0 + 1;
        if (j0 < 0 || j1 >= nz || nv < 1 || nv > SL) {
            if (threadIdx.x == 0) bflag(c);
            return;
        }
        const int64_t g0 = (int64_t)t * G, g1 = min(g0 + G, p.m);
        lds_barrier();
        // slice: row start | vertex | 1 if the vertex still misses a source
        for (int i = threadIdx.x; i < nv; i += kBlock) {
            const int v = p.nz_v[j0 + i];
            sl[i] = p.offsets[v];
            sl[SL + i] = v;
            bool need = false;
            unsigned long long vw[4];
            load_mask(p.vis + (int64_t)v * 4, vw);
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (w < W) need |= vw[w] != full[w];
            sl[2 * SL + i] = need;
#pragma unroll
            for (int w = 0; w < 4; ++w) lds.acc[i * 4 + w] = 0ull;
        }
        lds_barrier();
        int gg[BVT], own[BVT];
#pragma unroll
        for (int r = 0; r < BVT; ++r) gg[r] = (int)min(g0 + r * kBlock + (int64_t)threadIdx.x, g1 - 1);
        search_owners<BVT>(sl, nv, gg, own);
        // the neighbours of this lane's edges, then their activity, then their masks: each
        // step's loads for all BVT edges go out together, and the ORs into LDS come last
        int xs[BVT];
        bool open[BVT];
#pragma unroll
        for (int r = 0; r < BVT; ++r) {
            const int64_t g = g0 + r * kBlock + threadIdx.x;
            open[r] = g < g1 && sl[2 * SL + own[r]];
            xs[r] = open[r] ? (p.fr_hot ? p.colx[g] : p.cols[g]) : INT32_MAX;
        }
        uint32_t ab[BVT];
#pragma unroll
        for (int r = 0; r < BVT; ++r) {  // active bits from a clamped word, used only for x in [0, n)
            const int x = xs[r];
            ab[r] = p.act_bits[(x >= 0 && x < p.n ? x : 0) >> 5];
        }
        const unsigned long long* src[BVT];
#pragma unroll
        for (int r = 0; r < BVT; ++r) {
            const int x = xs[r];
            src[r] = nullptr;
            if (x < 0) {
                const int h = -1 - x;
                if (h < p.hot_count) src[r] = p.fr_hot + (int64_t)h * 4;
            } else if (x < p.n && ((ab[r] >> (x & 31)) & 1u)) {
                src[r] = p.fr + (int64_t)x * 4;
            }
        }
        unsigned long long f[BVT][4];
#pragma unroll
        for (int r = 0; r < BVT; ++r) {
            if (src[r]) load_mask(src[r], f[r]);
            else f[r][0] = f[r][1] = f[r][2] = f[r][3] = 0ull;
        }
#pragma unroll
        for (int r = 0; r < BVT; ++r) {
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (w < W && f[r][w]) atomicOr(&lds.acc[own[r] * 4 + w], f[r][w]);
        }
        lds_barrier();
        // hand the accumulated masks to N: rows cut by the sub-tile's ends may also be
        // accumulated by a neighbouring sub-tile, so those use atomics
        for (int i = threadIdx.x; i < nv; i += kBlock) {
            const int v = sl[SL + i];
            const int64_t r0 = sl[i], r1 = p.offsets[v + 1];
            const bool cut = r0 < g0 || r1 > g1;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if (w < W) {
                    const unsigned long long a = lds.acc[i * 4 + w];
                    if (a) {
                        if (cut) atomicOr(&p.nx[(int64_t)v * 4 + w], a);
                        else p.nx[(int64_t)v * 4 + w] = a;
                    }
                }
            }
        }
    }
}

template <int BVT>
__global__ void __launch_bounds__(kBlock) k_batch_expand(BatchParams p) {
    __shared__ ExpLds<BVT> lds;
    batch_expand<BVT>(p, blockIdx.x, gridDim.x, lds);
}

// Before a pull level: the masks of the hot vertices, in hot-number order, zero for those not
// active (the level whose expansion runs next is ctrl->blevel); thread `first` of `stride`.
__device__ __forceinline__ void batch_hotmask(const BatchParams& p, int64_t first, int64_t stride) {
    Ctrl* c = p.ctrl;
    if (!p.fr_hot || ld_acq(&c->bdone)) return;
    const int l = ld_acq(&c->blevel);
    if (ld_acq(&c->b_eact[l & 1]) <= p.args->pull_edges) return;  // a push level gathers nothing
    const int W = p.args->words;
    for (int64_t h = first; h < p.hot_count; h += stride) {
        const int v = p.hot_vid[h];
        const bool act = (unsigned)v < (unsigned)p.n && ((p.act_bits[v >> 5] >> (v & 31)) & 1u);
#pragma unroll
        for (int w = 0; w < 4; ++w)
            if (w < W) p.fr_hot[h * 4 + w] = act ? p.fr[(int64_t)v * 4 + w] : 0ull;
    }
}

__global__ void __launch_bounds__(kBlock) k_batch_hotmask(BatchParams p) {
    batch_hotmask(p, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// Advances the level; stops the loop when nothing is active or a level overflowed (one lane).
__device__ __forceinline__ void batch_next(const BatchParams& p) {
    Ctrl* c = p.ctrl;
    if (c->bdone) return;
    const int l = c->blevel + 1;
    c->blevel = l;
    const int na = c->b_nact[l & 1];
    if (na > 0) {
        if (l < kStatCap) {
            p.stat_nl[l] = na;
            p.stat_el[l] = c->b_eact[l & 1];
        }
        c->levels = l + 1;
    }
    if (na == 0 || c->batch_overflow || c->error) c->bdone = 1;
}

__global__ void k_batch_next(BatchParams p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) batch_next(p);
}

// The levels that the replays enqueued before it left, on one workgroup: expansion, the
// update tiles in index order, the level step and the hot masks, with a workgroup barrier
// between them.  Returns at once when the search has already stopped.  It needs no other
// workgroup to be resident, and it ends: every level either activates a vertex at a new
// depth, which stops at 255, or stops the loop.
template <int BVT, int UV>
__global__ void __launch_bounds__(kBlock) k_batch_finish(BatchParams p) {
    __shared__ union {
        ExpLds<BVT> e;
        UpdLds<UV> u;
    } lds;
    Ctrl* c = p.ctrl;
    for (;;) {
        __syncthreads();
        if (ld_acq(&c->bdone)) return;
        batch_expand<BVT>(p, 0, 1, lds.e);
        for (int t = 0; t < p.utiles; ++t) {
            __syncthreads();
            batch_update_tile<BVT, UV>(p, t, p.utiles, lds.u);
        }
        __syncthreads();
        if (threadIdx.x == 0) batch_next(p);
        __syncthreads();
        batch_hotmask(p, threadIdx.x, kBlock);
    }
}

// ---- host launchers ----------------------------------------------------------------------------

template <int BVT>
static const void* expand_kernel() {
    return reinterpret_cast<const void*>(k_batch_expand<BVT>);
}

int batch_grid_capacity(int device, int bvt) {
    const void* k = bvt == 1 ? expand_kernel<1>() : bvt == 4 ? expand_kernel<4>() : expand_kernel<2>();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, 0) != hipSuccess) return 0;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
    return per_cu * cus;
}

static int bfill_grid(int64_t items) {
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

static bool tiling_ok(const BatchParams& p) {
    return (p.bvt == 1 || p.bvt == 2 || p.bvt == 4) && (p.uv == 2 || p.uv == 4 || p.uv == 8);
}

template <int BVT>
static void launch_nz(const BatchParams& p, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_nz<BVT>, dim3((p.n + kNzTile - 1) / kNzTile), dim3(kBlock), 0, s, p);
}

template <int BVT, int UV>
static void launch_update_t(const BatchParams& p, hipStream_t s) {
    hipLaunchKernelGGL((k_batch_update<BVT, UV>), dim3(p.utiles), dim3(kBlock), 0, s, p);
}

template <int BVT>
static void launch_update_b(const BatchParams& p, hipStream_t s) {
    if (p.uv == 2) launch_update_t<BVT, 2>(p, s);
    else if (p.uv == 8) launch_update_t<BVT, 8>(p, s);
    else launch_update_t<BVT, 4>(p, s);
}

static void launch_update(const BatchParams& p, hipStream_t s) {
    if (p.bvt == 1) launch_update_b<1>(p, s);
    else if (p.bvt == 4) launch_update_b<4>(p, s);
    else launch_update_b<2>(p, s);
}

static void launch_expand(const BatchParams& p, int grid, hipStream_t s) {
    if (p.bvt == 1) hipLaunchKernelGGL(k_batch_expand<1>, dim3(grid), dim3(kBlock), 0, s, p);
    else if (p.bvt == 4) hipLaunchKernelGGL(k_batch_expand<4>, dim3(grid), dim3(kBlock), 0, s, p);
    else hipLaunchKernelGGL(k_batch_expand<2>, dim3(grid), dim3(kBlock), 0, s, p);
}

// Per grain: the list of vertices of degree >= 1 and its sub-tile starts.
hipError_t launch_batch_setup(const BatchParams& p, int grid, hipStream_t s) {
    (void)grid;
    if (!tiling_ok(p)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_prep, dim3(bfill_grid(p.n)), dim3(kBlock), 0, s, p);
    if (p.bvt == 1) launch_nz<1>(p, s);
    else if (p.bvt == 4) launch_nz<4>(p, s);
    else launch_nz<2>(p, s);
    return hipGetLastError();
}

// A run's arguments, passed by value: each launch carries its own copy, so calls queued back to
// back on one stream cannot see each other's.
__global__ void k_batch_args(BatchArgs* dst, BatchArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = a;
}

hipError_t launch_batch_args(BatchArgs* dst, const BatchArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_args, dim3(1), dim3(64), 0, s, dst, a);
    return hipGetLastError();
}

// Per run: reset, seed, and the update that turns the seeds into level 0.
hipError_t launch_batch_start(const BatchParams& p, hipStream_t s) {
    if (!tiling_ok(p)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_prep, dim3(bfill_grid((int64_t)p.n * 4)), dim3(kBlock), 0, s, p);
    hipLaunchKernelGGL(k_batch_seed, dim3(1), dim3(64), 0, s, p);
    launch_update(p, s);
    hipLaunchKernelGGL(k_batch_next, dim3(1), dim3(64), 0, s, p);
    if (p.fr_hot) hipLaunchKernelGGL(k_batch_hotmask, dim3(bfill_grid(p.hot_count)), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

template <int BVT>
static void launch_finish_b(const BatchParams& p, hipStream_t s) {
    if (p.uv == 2) hipLaunchKernelGGL((k_batch_finish<BVT, 2>), dim3(1), dim3(kBlock), 0, s, p);
    else if (p.uv == 8) hipLaunchKernelGGL((k_batch_finish<BVT, 8>), dim3(1), dim3(kBlock), 0, s, p);
    else hipLaunchKernelGGL((k_batch_finish<BVT, 4>), dim3(1), dim3(kBlock), 0, s, p);
}

// Whatever levels remain after the replays, on one workgroup (a no-op once the loop stopped).
hipError_t launch_batch_finish(const BatchParams& p, hipStream_t s) {
    if (!tiling_ok(p)) return hipErrorInvalidValue;
    if (p.bvt == 1) launch_finish_b<1>(p, s);
    else if (p.bvt == 4) launch_finish_b<4>(p, s);
    else launch_finish_b<2>(p, s);
    return hipGetLastError();
}

// One level: expand, update, next (captured into a graph by the caller).
hipError_t launch_batch_level(const BatchParams& p, int grid, hipStream_t s) {
    if (!tiling_ok(p)) return hipErrorInvalidValue;
    launch_expand(p, grid, s);
    launch_update(p, s);
    hipLaunchKernelGGL(k_batch_next, dim3(1), dim3(64), 0, s, p);
    if (p.fr_hot) hipLaunchKernelGGL(k_batch_hotmask, dim3(bfill_grid(p.hot_count)), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

}  // namespace s3bfs
