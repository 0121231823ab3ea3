/*
 * CPU oracle for breadth-first search.  TEST INFRASTRUCTURE ONLY: used by
 * the tests, by the harness's smoke check and by the benchmark's CPU
 * baseline leg, never by the GPU library.  It shares no code with it.
 *
 * What it computes is the plain definition of the result of the paper's
 * Parallel-BFS(s, P) (Figure 1, whose header says it returns d[0:n-1], the
 * distance of every vertex from s; the Introduction defines the
 * level-synchronous traversal):
 *   level[v]  = hop distance from the source, -1 if v is unreachable
 *               (the paper's "infinity");
 *   parent[v] = the smallest-id neighbour u of v with level[u] = level[v]-1
 *               for a reached v that is not a root, parent[root] = root,
 *               and -1 for an unreached v.  The paper defines no parent;
 *               this deterministic rule makes parents comparable bit for bit.
 * With several roots the distance is to the nearest root (one root per
 * component gives independent searches of a disjoint union of graphs).
 *
 * The algorithm is a sequential FIFO-queue BFS (first-in first-out order
 * visits vertices in non-decreasing distance, so the first time a vertex
 * is seen fixes its distance), then a separate parent pass that scans every
 * neighbour of every reached vertex: it does not rely on sorted rows, on
 * early exit or on the order of discovery.
 */
#include <stdint.h>
#include <stdlib.h>

/* Returns the number of levels (max level + 1), 0 if there are no roots,
   -1 if a root is out of range, -2 if memory runs out. */
int32_t oracle_bfs_levels(int32_t n, const int32_t* offsets, const int32_t* cols,
                          int32_t nroots, const int32_t* roots, int32_t* level) {
    for (int32_t i = 0; i < nroots; ++i)
        if (roots[i] < 0 || roots[i] >= n) return -1;
    for (int32_t v = 0; v < n; ++v) level[v] = -1;
    if (nroots == 0) return 0;
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!queue) return -2;
    int64_t head = 0, tail = 0;
    for (int32_t i = 0; i < nroots; ++i) {
        int32_t r = roots[i];
        if (level[r] == -1) {
            level[r] = 0;
            queue[tail++] = r;
        }
    }
    int32_t maxlev = 0;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
            int32_t v = cols[e];
            if (level[v] == -1) {
                level[v] = level[u] + 1;
                if (level[v] > maxlev) maxlev = level[v];
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return maxlev + 1;
}

/* parent[] from level[]: smallest-id neighbour one level up; roots
   (level 0) point to themselves; unreached vertices get -1. */
void oracle_parents(int32_t n, const int32_t* offsets, const int32_t* cols,
                    const int32_t* level, int32_t* parent) {
    for (int32_t v = 0; v < n; ++v) {
        if (level[v] < 0) { parent[v] = -1; continue; }
        if (level[v] == 0) { parent[v] = v; continue; }
        int32_t best = -1;
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
            int32_t u = cols[e];
            if (level[u] == level[v] - 1 && (best == -1 || u < best)) best = u;
        }
        parent[v] = best;
    }
}

int32_t oracle_bfs(int32_t n, const int32_t* offsets, const int32_t* cols,
                   int32_t nroots, const int32_t* roots, int32_t* level, int32_t* parent) {
    int32_t rc = oracle_bfs_levels(n, offsets, cols, nroots, roots, level);
    if (rc < 0) return rc;
    if (parent) oracle_parents(n, offsets, cols, level, parent);
    return rc;
}

/* k single-source searches; out[v * k + j] = level of v from sources[j]
   as uint8, 255 when unreached.  Returns 1 if some level is >= 255 (it
   does not fit; such entries hold 255 too), 0 otherwise, <0 on error. */
int32_t oracle_bfs_batch_u8(int32_t n, const int32_t* offsets, const int32_t* cols,
                            int32_t k, const int32_t* sources, uint8_t* out) {
    int32_t* level = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!level) return -2;
    int32_t overflow = 0;
    for (int32_t j = 0; j < k; ++j) {
        int32_t rc = oracle_bfs_levels(n, offsets, cols, 1, &sources[j], level);
        if (rc < 0) { free(level); return rc; }
        for (int32_t v = 0; v < n; ++v) {
            int32_t l = level[v];
            if (l >= 255) overflow = 1;
            out[(int64_t)v * k + j] = (uint8_t)((l < 0 || l >= 255) ? 255 : l);
        }
    }
    free(level);
    return overflow;
}
