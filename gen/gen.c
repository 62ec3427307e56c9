/*
 * Seeded synthetic input generators: R-MAT and Erdos-Renyi edge sets, a random
 * vertex relabelling, de-duplication into a sorted CSR, per-edge weights and
 * source vertices.
 *
 * This module produces inputs only. It holds none of the graph-processing
 * method's arithmetic, and both the GPU library and the CPU oracle consume its
 * output.
 *
 * Randomness is counter based: draw number c of stream `seed` is
 *     mix64(mix64(seed) + c * 0x9E3779B97F4A7C15)
 * where mix64 is the SplitMix64 output function (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014). Every output
 * is therefore a pure function of (seed, counter), independent of the number of
 * threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t seed_key, uint64_t counter) {
    return mix64(seed_key + counter * 0x9E3779B97F4A7C15ull);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* Uniform integer in [0, bound) by 128-bit multiply-shift (Lemire's method). */
static inline uint64_t below(uint64_t r, uint64_t bound) {
    return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

uint64_t gen_draw(uint64_t seed, uint64_t counter) { return draw(mix64(seed), counter); }

/*
 * R-MAT (Chakrabarti, Zhan & Faloutsos, SDM 2004): edge i descends `scale`
 * levels of the adjacency matrix; at level l it picks quadrant
 *   a -> (row 0, col 0), b -> (0, 1), c -> (1, 0), d -> (1, 1)
 * with draw counter i * 64 + l. No noise is added.
 */
void gen_rmat_edges(int scale, uint64_t m, double a, double b, double c, uint64_t seed,
                    uint32_t* src, uint32_t* dst) {
    const uint64_t key = mix64(seed);
    const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        uint32_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            double r = unit(draw(key, (uint64_t)i * 64u + (uint64_t)l));
            uint32_t rb, cb;
            if (r < a) { rb = 0; cb = 0; }
            else if (r < ab) { rb = 0; cb = 1; }
            else if (r < abc) { rb = 1; cb = 0; }
            else { rb = 1; cb = 1; }
            u = (u << 1) | rb;
            v = (v << 1) | cb;
        }
        src[i] = u;
        dst[i] = v;
    }
}

/* Uniform directed pairs over [0, n) x [0, n): edge i uses counters 2i and 2i+1. */
void gen_uniform_edges(uint32_t n, uint64_t m, uint64_t seed, uint64_t first, uint32_t* src,
                       uint32_t* dst) {
    const uint64_t key = mix64(seed);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        uint64_t c = ((uint64_t)i + first) * 2u;
        src[i] = (uint32_t)below(draw(key, c), n);
        dst[i] = (uint32_t)below(draw(key, c + 1), n);
    }
}

/* Fisher-Yates shuffle of the identity, step j drawing counter j. */
void gen_permutation(uint32_t n, uint64_t seed, uint32_t* perm) {
    const uint64_t key = mix64(seed);
    for (uint32_t i = 0; i < n; ++i) perm[i] = i;
    for (uint64_t j = n; j > 1; --j) {
        uint64_t k = below(draw(key, j), j);
        uint32_t t = perm[j - 1];
        perm[j - 1] = perm[k];
        perm[k] = t;
    }
}

void gen_apply_permutation(uint64_t m, const uint32_t* perm, uint32_t* src, uint32_t* dst) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        src[i] = perm[src[i]];
        dst[i] = perm[dst[i]];
    }
}

static int cmp_u64(const void* x, const void* y) {
    uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
    return (a > b) - (a < b);
}

/*
 * Build a CSR with rows sorted by neighbour id, self-loops and duplicate pairs
 * removed. When `tag` is non-null it carries one 32-bit tag per input edge and
 * duplicates keep the smallest tag (used to keep the earliest-drawn copy);
 * tag_out then receives the surviving tags in CSR order.
 * col_out must hold m entries; returns the number of edges kept.
 */
uint64_t gen_build_csr(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                       const uint32_t* tag, uint64_t* row_off, uint32_t* col_out,
                       uint32_t* tag_out) {
    uint64_t* cnt = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        if (src[i] != dst[i]) {
#pragma omp atomic
            cnt[src[i] + 1]++;
        }
    }
    for (uint32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    uint64_t total = cnt[n];
    /* key = (neighbour << 32) | tag, so sorting a row orders by neighbour then tag */
    uint64_t* keys = (uint64_t*)malloc((size_t)(total ? total : 1) * sizeof(uint64_t));
    uint64_t* cur = (uint64_t*)malloc(((size_t)n + 1) * sizeof(uint64_t));
    memcpy(cur, cnt, ((size_t)n + 1) * sizeof(uint64_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)m; ++i) {
        if (src[i] == dst[i]) continue;
        uint64_t slot;
#pragma omp atomic capture
        slot = cur[src[i]]++;
        keys[slot] = ((uint64_t)dst[i] << 32) | (tag ? tag[i] : 0u);
    }
    free(cur);
    uint32_t* kept = (uint32_t*)calloc((size_t)n + 1, sizeof(uint32_t));
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t u = 0; u < (int64_t)n; ++u) {
        uint64_t b = cnt[u], e = cnt[u + 1];
        if (e - b > 1) qsort(keys + b, e - b, sizeof(uint64_t), cmp_u64);
        uint64_t w = b;
        for (uint64_t j = b; j < e; ++j)
            if (j == b || (keys[j] >> 32) != (keys[w - 1] >> 32)) keys[w++] = keys[j];
        kept[u] = (uint32_t)(w - b);
    }
    row_off[0] = 0;
    for (uint32_t u = 0; u < n; ++u) row_off[u + 1] = row_off[u] + kept[u];
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t u = 0; u < (int64_t)n; ++u) {
        uint64_t b = cnt[u], o = row_off[u];
        for (uint32_t j = 0; j < kept[u]; ++j) {
            col_out[o + j] = (uint32_t)(keys[b + j] >> 32);
            if (tag_out) tag_out[o + j] = (uint32_t)keys[b + j];
        }
    }
    uint64_t out = row_off[n];
    free(kept);
    free(keys);
    free(cnt);
    return out;
}

/* Keep, row by row, only edges whose tag is < cutoff; compacts in place. */
uint64_t gen_filter_tag_below(uint32_t n, uint64_t* row_off, uint32_t* col, const uint32_t* tag,
                              uint32_t cutoff) {
    uint64_t w = 0, b = 0;
    for (uint32_t u = 0; u < n; ++u) {
        uint64_t e = row_off[u + 1];
        for (uint64_t j = b; j < e; ++j)
            if (tag[j] < cutoff) col[w++] = col[j];
        b = e;
        row_off[u + 1] = w;
    }
    return w;
}

/* w(u, v) = lo + mix64(mix64(seed) ^ (u << 32 | v)) mod (hi - lo + 1): a function of the edge. */
void gen_edge_weights(uint32_t n, const uint64_t* row_off, const uint32_t* col, uint64_t seed,
                      uint32_t lo, uint32_t hi, uint32_t* w) {
    const uint64_t key = mix64(seed);
    const uint64_t span = (uint64_t)hi - lo + 1;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < (int64_t)n; ++u)
        for (uint64_t j = row_off[u]; j < row_off[u + 1]; ++j)
            w[j] = lo + (uint32_t)(mix64(key ^ (((uint64_t)u << 32) | col[j])) % span);
}

/* Draw vertices uniformly (counter j for the j-th try), keeping those with out-degree >= 1. */
int gen_pick_sources(uint32_t n, const uint64_t* row_off, uint32_t count, uint64_t seed,
                     uint32_t* out) {
    const uint64_t key = mix64(seed);
    uint32_t got = 0;
    for (uint64_t j = 0; got < count && j < 64ull * n + 1024; ++j) {
        uint32_t v = (uint32_t)below(draw(key, j), n);
        if (row_off[v + 1] > row_off[v]) out[got++] = v;
    }
    return got == count ? 0 : -1;
}

int gen_threads(void) { return omp_get_max_threads(); }
