/*
 * Seeded synthetic graph generators (input generation only).
 *
 * Nothing in this file computes a breadth-first search or any step of one:
 * it only produces symmetric CSR graphs and source lists that both the CPU
 * oracle and the GPU library consume.
 *
 * Randomness is counter based: every draw is a pure function of
 * (seed, stream, counter), computed with the SplitMix64 output mix
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014).  Results therefore do not depend on the thread count.
 *
 * Graph families (the paper names none precisely; these stand in for its
 * real-world and synthetic graphs):
 *   R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004): EF * 2^S samples,
 *     one 64-bit draw per (sample, bit) compared with integer thresholds
 *     for the quadrant probabilities a, a+b, a+b+c; quadrant a -> (0,0),
 *     b -> (0,1), c -> (1,0), d -> (1,1); then a seeded vertex permutation.
 *   2-D 4-neighbour grid, id = r * W + c.
 *   Erdos-Renyi G(n, M): M uniform vertex pairs.
 *   Power-law forest: 64 roots, vertex i >= 64 attaches to an earlier vertex
 *     chosen with probability proportional to (degree + 1).
 * Every edge list goes through the same CSR builder: self-loops dropped,
 * both directions added, rows sorted ascending, duplicates removed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

static inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* One 64-bit draw keyed by (seed, stream, counter). */
static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t counter) {
    return mix64(mix64(seed ^ mix64(stream)) ^ counter);
}

/* Uniform integer in [0, bound) by the multiply-high method. */
static inline uint64_t below(uint64_t r, uint64_t bound) {
    return (uint64_t)(((__uint128_t)r * (__uint128_t)bound) >> 64);
}

uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t counter) {
    return draw(seed, stream, counter);
}

static uint64_t prob_threshold(double p) {
    if (p <= 0.0) return 0;
    if (p >= 1.0) return UINT64_MAX;
    long double t = ldexpl((long double)p, 64);
    return (uint64_t)t;
}

/* Seeded permutation of [0, n) by Fisher-Yates. */
void gg_permutation(int32_t n, uint64_t seed, int32_t* perm) {
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int64_t i = (int64_t)n - 1; i > 0; --i) {
        int64_t j = (int64_t)below(draw(seed, 7, (uint64_t)i), (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/* R-MAT edge samples: src/dst each of length ef << scale. */
void gg_rmat_samples(int32_t scale, int32_t edgefactor, double a, double b, double c,
                     uint64_t seed, int permute, uint64_t perm_seed,
                     int32_t* src, int32_t* dst) {
    const int64_t n = (int64_t)1 << scale;
    const int64_t M = (int64_t)edgefactor * n;
    const uint64_t ta = prob_threshold(a), tab = prob_threshold(a + b), tabc = prob_threshold(a + b + c);
    int32_t* perm = NULL;
    if (permute) {
        perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        gg_permutation((int32_t)n, perm_seed, perm);
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        uint32_t u = 0, v = 0;
        for (int32_t bit = 0; bit < scale; ++bit) {
            uint64_t r = draw(seed, 1, ((uint64_t)i << 6) | (uint64_t)bit);
            uint32_t qu, qv;
            if (r < ta) { qu = 0; qv = 0; }
            else if (r < tab) { qu = 0; qv = 1; }
            else if (r < tabc) { qu = 1; qv = 0; }
            else { qu = 1; qv = 1; }
            u = (u << 1) | qu;
            v = (v << 1) | qv;
        }
        if (perm) { u = (uint32_t)perm[u]; v = (uint32_t)perm[v]; }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
    free(perm);
}

/* Uniform vertex pairs for G(n, M). */
void gg_er_samples(int32_t n, int64_t M, uint64_t seed, int32_t* src, int32_t* dst) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        src[i] = (int32_t)below(draw(seed, 2, 2 * (uint64_t)i), (uint64_t)n);
        dst[i] = (int32_t)below(draw(seed, 2, 2 * (uint64_t)i + 1), (uint64_t)n);
    }
}

/* Preferential-attachment forest: n - nroots edges, returned as (src, dst). */
void gg_forest_samples(int32_t n, int32_t nroots, uint64_t seed, int32_t* src, int32_t* dst) {
    /* urn holds each vertex once plus once per incident edge, so a uniform
       pick from it is proportional to degree + 1 */
    int64_t cap = (int64_t)n + 2 * (int64_t)n;
    int32_t* urn = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    int64_t len = 0;
    for (int32_t i = 0; i < nroots && i < n; ++i) urn[len++] = i;
    int64_t e = 0;
    for (int32_t i = nroots; i < n; ++i) {
        int32_t t = urn[below(draw(seed, 3, (uint64_t)i), (uint64_t)len)];
        src[e] = i; dst[e] = t; ++e;
        urn[len++] = i;
        urn[len++] = i;
        urn[len++] = t;
    }
    free(urn);
}

static int cmp_i32(const void* x, const void* y) {
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

/*
 * Symmetric, sorted, deduplicated CSR from M (src, dst) samples, in two
 * calls.  gg_csr_build returns the number of directed entries m and keeps
 * the built rows in an internal handle *work; the caller allocates
 * offsets[n+1] and cols[m] and gg_csr_emit copies the rows out and frees
 * the handle (it returns -1 if m does not fit in int32).
 */
typedef struct { int64_t n; int64_t* off; int32_t* cols; int64_t* newdeg; } gg_build_t;

int64_t gg_csr_build(int32_t n, int64_t M, const int32_t* src, const int32_t* dst, void** work) {
    gg_build_t* w = (gg_build_t*)calloc(1, sizeof(gg_build_t));
    w->n = n;
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        int32_t u = src[i], v = dst[i];
        if (u == v) continue;
        __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
    }
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) off[v + 1] = off[v] + cnt[v];
    int64_t total = off[n];
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    for (int64_t v = 0; v < n; ++v) cnt[v] = off[v];
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        int32_t u = src[i], v = dst[i];
        if (u == v) continue;
        int64_t pu = __atomic_fetch_add(&cnt[u], 1, __ATOMIC_RELAXED);
        int64_t pv = __atomic_fetch_add(&cnt[v], 1, __ATOMIC_RELAXED);
        tmp[pu] = v;
        tmp[pv] = u;
    }
    int64_t* newdeg = cnt; /* reuse */
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < n; ++v) {
        int32_t* row = tmp + off[v];
        int64_t d = off[v + 1] - off[v];
        if (d > 1) qsort(row, (size_t)d, sizeof(int32_t), cmp_i32);
        int64_t k = 0;
        for (int64_t j = 0; j < d; ++j)
            if (k == 0 || row[j] != row[k - 1]) row[k++] = row[j];
        newdeg[v] = k;
    }
    w->off = off; w->cols = tmp; w->newdeg = newdeg;
    int64_t m = 0;
    for (int64_t v = 0; v < n; ++v) m += newdeg[v];
    *work = w;
    return m;
}

int gg_csr_emit(void* work, int32_t* offsets, int32_t* cols) {
    gg_build_t* w = (gg_build_t*)work;
    int64_t n = w->n;
    int64_t acc = 0;
    int rc = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (acc > INT32_MAX) { rc = -1; break; }
        offsets[v] = (int32_t)acc;
        acc += w->newdeg[v];
    }
    if (acc > INT32_MAX) rc = -1;
    if (rc == 0) {
        offsets[n] = (int32_t)acc;
        #pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t v = 0; v < n; ++v)
            memcpy(cols + offsets[v], w->cols + w->off[v], sizeof(int32_t) * (size_t)w->newdeg[v]);
    }
    free(w->off); free(w->cols); free(w->newdeg); free(w);
    return rc;
}

/* W x H 4-neighbour grid; each row lists up, left, right, down (ascending ids). */
int64_t gg_grid_m(int32_t W, int32_t H) {
    if (W <= 0 || H <= 0) return 0;
    return 2 * ((int64_t)(W - 1) * H + (int64_t)W * (H - 1));
}

void gg_grid(int32_t W, int32_t H, int32_t* offsets, int32_t* cols) {
    int64_t n = (int64_t)W * H;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < H; ++r) {
        /* directed entries in rows < r: each row has 2(W-1) horizontal ones,
           W upward ones if it is not the first row, W downward ones if it is
           not the last */
        int64_t horiz = (W > 1) ? 2 * (int64_t)(W - 1) : 0;
        int64_t ups = r > 0 ? r - 1 : 0;
        int64_t downs = r < H - 1 ? r : H - 1;
        int64_t acc = r * horiz + (int64_t)W * (ups + downs);
        int64_t pos = acc;
        for (int64_t c = 0; c < W; ++c) {
            int64_t id = r * W + c;
            offsets[id] = (int32_t)pos;
            if (r > 0) cols[pos++] = (int32_t)(id - W);
            if (c > 0) cols[pos++] = (int32_t)(id - 1);
            if (c < W - 1) cols[pos++] = (int32_t)(id + 1);
            if (r < H - 1) cols[pos++] = (int32_t)(id + W);
        }
    }
    offsets[n] = (int32_t)gg_grid_m(W, H);
}

/*
 * k sources drawn uniformly among vertices with degree >= 1.
 * distinct != 0 draws without replacement (k must not exceed their count).
 * Returns the number of eligible vertices, or -1 if there are not enough.
 */
int64_t gg_pick_sources(int32_t n, const int32_t* offsets, uint64_t seed, int32_t k,
                        int distinct, int32_t* out) {
    int32_t* elig = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t ne = 0;
    for (int32_t v = 0; v < n; ++v)
        if (offsets[v + 1] > offsets[v]) elig[ne++] = v;
    if (ne == 0 || (distinct && k > ne)) { free(elig); return -1; }
    uint64_t ctr = 0;
    for (int32_t i = 0; i < k; ++i) {
        for (;;) {
            int32_t cand = elig[below(draw(seed, 4, ctr++), (uint64_t)ne)];
            int dup = 0;
            if (distinct)
                for (int32_t j = 0; j < i; ++j)
                    if (out[j] == cand) { dup = 1; break; }
            if (!dup) { out[i] = cand; break; }
        }
    }
    free(elig);
    return ne;
}

int gg_num_threads(void) { return omp_get_max_threads(); }
