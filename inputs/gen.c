/*
 * Seeded synthetic input generators shared by the CPU oracle and the GPU path.
 *
 * This file holds no arithmetic of the task-parallel method itself: it only
 * draws random numbers and lays out the workloads (uniform sort keys, R-MAT
 * graphs in CSR form) that the method is then run on.
 *
 * Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used counter-based:
 * draw(seed, i) is the (i+1)-th output of a SplitMix64 stream whose state
 * starts at `seed`, so any draw can be computed independently (and in
 * parallel) from (seed, i).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SM64_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t tin_mix(uint64_t z) { return sm64_mix(z); }

uint64_t tin_draw(uint64_t seed, uint64_t i) {
    return sm64_mix(seed + (i + 1) * SM64_GAMMA);
}

/* Uniform integer in [lo, hi] from the high 32 bits of one draw. */
static inline int64_t uni(uint64_t seed, uint64_t i, int64_t lo, int64_t hi) {
    uint64_t x = tin_draw(seed, i) >> 32;
    uint64_t span = (uint64_t)(hi - lo + 1);
    return lo + (int64_t)((x * span) >> 32);
}

int64_t tin_uniform(uint64_t seed, uint64_t i, int64_t lo, int64_t hi) {
    return uni(seed, i, lo, hi);
}

/* out[i] = high 32 bits of draw(seed, i): keys uniform over [0, 2^32). */
void tin_keys_u32(uint64_t seed, int64_t n, uint32_t *out) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = (uint32_t)(tin_draw(seed, (uint64_t)i) >> 32);
}

/* Fisher-Yates shuffle of 0..n-1; step k (k = n-1 .. 1) swaps k with
 * uniform[0, k] taken from draw index (n-1-k). */
void tin_permutation(uint64_t seed, int64_t n, int32_t *perm) {
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t k = n - 1; k >= 1; --k) {
        int64_t j = uni(seed, (uint64_t)(n - 1 - k), 0, k);
        int32_t t = perm[k]; perm[k] = perm[j]; perm[j] = t;
    }
}

/* A random binary tree of n nodes rooted at node 0: node v (v = 1..n-1)
 * becomes a child of node p = uniform[0, v-1] on side s = uniform[0, 1]
 * (0 = left), taken from draw indices v*64 + k and v*64 + k + 32 for the
 * k-th try; a try whose slot is taken is redrawn.  -1 = no child. */
void tin_binary_tree(uint64_t seed, int64_t n, int32_t *left, int32_t *right) {
    for (int64_t v = 0; v < n; ++v) left[v] = right[v] = -1;
    for (int64_t v = 1; v < n; ++v) {
        for (uint64_t k = 0;; ++k) {
            const int64_t p = uni(seed, (uint64_t)v * 64 + k, 0, v - 1);
            int32_t *side = uni(seed, (uint64_t)v * 64 + k + 32, 0, 1) == 0 ? left : right;
            if (side[p] == -1) { side[p] = (int32_t)v; break; }
        }
    }
}

/*
 * R-MAT edge list (Chakrabarti, Zhan, Faloutsos, SDM 2004).  Edge j descends
 * `scale` quadrant levels, most significant bit first.  Level l uses one
 * 32-bit half of draw index j*ceil(scale/2) + l/2 (high half for even l, low
 * half for odd l), compared against the cumulative thresholds thr[0..2]
 * (a, a+b, a+b+c scaled to 2^32).  Quadrant 0: (0,0), 1: (0,1), 2: (1,0),
 * 3: (1,1) for the (source bit, destination bit) pair.
 */
void tin_rmat_edges(int32_t scale, int64_t nedges, uint64_t seed,
                    const uint32_t *thr, int32_t *src, int32_t *dst) {
    const int64_t per = (scale + 1) / 2;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nedges; ++j) {
        uint32_t s = 0, d = 0;
        uint64_t x = 0;
        for (int32_t l = 0; l < scale; ++l) {
            if ((l & 1) == 0) x = tin_draw(seed, (uint64_t)(j * per + l / 2));
            uint32_t r = (l & 1) ? (uint32_t)x : (uint32_t)(x >> 32);
            uint32_t q = (r < thr[0]) ? 0u : (r < thr[1]) ? 1u : (r < thr[2]) ? 2u : 3u;
            uint32_t bit = 1u << (scale - 1 - l);
            if (q & 2u) s |= bit;
            if (q & 1u) d |= bit;
        }
        src[j] = (int32_t)s;
        dst[j] = (int32_t)d;
    }
}

/* Apply a vertex relabelling in place: v -> perm[v]. */
void tin_relabel(int64_t n, const int32_t *perm, int32_t *v) {
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) v[j] = perm[v[j]];
}

/*
 * Stable counting sort of the arc list by source: row_ptr[V+1] and
 * col_idx[E] (arcs of one source keep their edge-list order).
 */
void tin_csr(int64_t V, int64_t E, const int32_t *src, const int32_t *dst,
             int32_t *row_ptr, int32_t *col_idx) {
    int64_t *cnt = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
    for (int64_t j = 0; j < E; ++j) cnt[src[j] + 1]++;
    for (int64_t v = 0; v < V; ++v) cnt[v + 1] += cnt[v];
    for (int64_t v = 0; v <= V; ++v) row_ptr[v] = (int32_t)cnt[v];
    for (int64_t j = 0; j < E; ++j) col_idx[cnt[src[j]]++] = dst[j];
    free(cnt);
}
