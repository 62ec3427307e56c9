/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately simple reference for the Wedge pull-only
 * frontier method (Grossman & Kozyrakis, "A New Frontier for Pull-Based Graph
 * Processing", arXiv 1903.07754). Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may call it; the GPU library never does, and the
 * two share no code.
 *
 * Contents
 *   - plain definitions of the four results:
 *       or_bfs_levels    BFS hop levels (queue BFS)
 *       or_wcc_labels    weakly connected components, min-id label (union-find)
 *       or_sssp_dist     single-source shortest paths (Dijkstra / Dial buckets)
 *       or_pagerank      PageRank power iteration in FP64, compensated sums
 *   - the method's per-iteration behaviour, written from the paper:
 *       or_pull_engine   synchronous pull engine that consumes only the active
 *                        subset, with the frontier-fullness decision, the
 *                        Wedge Frontier size and per-iteration trace
 *       or_push_engine   textbook frontier-driven push engine (same iteration
 *                        semantics), used as an independent cross-check
 *       or_wedge_frontier  Wedge Frontier of a vertex frontier by a full scan of
 *                        the in-edge array
 *   - helpers: CSC from CSR (counting sort), undirected view of a CSR.
 *
 * Iteration semantics: the paper processes synchronously, in two phases that
 * all vertices finish before the next starts (Background, first paragraph).
 * Iteration k therefore reads the values left by iteration k-1 and writes new
 * ones; a vertex joins the next frontier exactly when its value is updated
 * (Background, Push vs. Pull).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define INF32 0xFFFFFFFFu

enum { APP_BFS = 1, APP_CC = 2, APP_SSSP = 3 };

/* ---------------------------------------------------------------- helpers */

/*
 * In-edge (CSC) form of a CSR (Background, Graph Representation): vertex index
 * col_off[n+1] and edge array in_src[m], grouped by destination. Edges are
 * scattered in CSR order, so within each destination the sources ascend.
 * in_w receives the weight of each in-edge when w is non-null.
 */
void or_csc_from_csr(uint32_t n, const uint64_t* row_off, const uint32_t* col, const uint32_t* w,
                     uint64_t* col_off, uint32_t* in_src, uint32_t* in_w) {
    uint64_t m = row_off[n];
    memset(col_off, 0, ((size_t)n + 1) * sizeof(uint64_t));
    for (uint64_t q = 0; q < m; ++q) col_off[col[q] + 1]++;
    for (uint32_t v = 0; v < n; ++v) col_off[v + 1] += col_off[v];
    uint64_t* cur = (uint64_t*)malloc(((size_t)n + 1) * sizeof(uint64_t));
    memcpy(cur, col_off, ((size_t)n + 1) * sizeof(uint64_t));
    for (uint32_t u = 0; u < n; ++u) {
        for (uint64_t q = row_off[u]; q < row_off[u + 1]; ++q) {
            uint64_t p = cur[col[q]]++;
            in_src[p] = u;
            if (w && in_w) in_w[p] = w[q];
        }
    }
    free(cur);
}

static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

/*
 * Undirected view: every edge u->v (u != v) contributes u->v and v->u;
 * duplicates are merged. out_col must hold 2*m entries. Returns the edge count.
 */
uint64_t or_symmetrize(uint32_t n, const uint64_t* row_off, const uint32_t* col,
                       uint64_t* out_row_off, uint32_t* out_col) {
    uint64_t m = row_off[n];
    uint64_t* deg = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t q = row_off[u]; q < row_off[u + 1]; ++q)
            if (col[q] != u) { deg[u + 1]++; deg[col[q] + 1]++; }
    for (uint32_t v = 0; v < n; ++v) deg[v + 1] += deg[v];
    uint64_t* cur = (uint64_t*)malloc(((size_t)n + 1) * sizeof(uint64_t));
    memcpy(cur, deg, ((size_t)n + 1) * sizeof(uint64_t));
    uint32_t* tmp = (uint32_t*)malloc((size_t)(2 * m + 1) * sizeof(uint32_t));
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t q = row_off[u]; q < row_off[u + 1]; ++q)
            if (col[q] != u) { tmp[cur[u]++] = col[q]; tmp[cur[col[q]]++] = u; }
    uint64_t out = 0;
    out_row_off[0] = 0;
    for (uint32_t u = 0; u < n; ++u) {
        uint64_t b = deg[u], e = deg[u + 1];
        qsort(tmp + b, e - b, sizeof(uint32_t), cmp_u32);
        for (uint64_t j = b; j < e; ++j)
            if (j == b || tmp[j] != tmp[j - 1]) out_col[out++] = tmp[j];
        out_row_off[u + 1] = out;
    }
    free(tmp); free(cur); free(deg);
    return out;
}

/* ------------------------------------------------- plain result definitions */

/*
 * BFS (Evaluation, Applications): level[v] = fewest edges on a directed path
 * src -> v, INF32 when unreachable. Textbook FIFO queue.
 */
void or_bfs_levels(uint32_t n, const uint64_t* row_off, const uint32_t* col, uint32_t src,
                   uint32_t* level) {
    for (uint32_t v = 0; v < n; ++v) level[v] = INF32;
    if (src >= n) return;
    uint32_t* q = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    uint64_t head = 0, tail = 0;
    level[src] = 0;
    q[tail++] = src;
    while (head < tail) {
        uint32_t u = q[head++];
        for (uint64_t j = row_off[u]; j < row_off[u + 1]; ++j) {
            uint32_t v = col[j];
            if (level[v] == INF32) { level[v] = level[u] + 1; q[tail++] = v; }
        }
    }
    free(q);
}

static uint32_t uf_find(uint32_t* parent, uint32_t x) {
    while (parent[x] != x) { parent[x] = parent[parent[x]]; x = parent[x]; }
    return x;
}

/*
 * CC (Evaluation, Applications: HCC label propagation). HCC's fixed point on
 * the undirected view is the smallest vertex id of each weakly connected
 * component; computed here by union-find that always keeps the smaller root.
 */
void or_wcc_labels(uint32_t n, const uint64_t* row_off, const uint32_t* col, uint32_t* label) {
    uint32_t* parent = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    for (uint32_t v = 0; v < n; ++v) parent[v] = v;
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t j = row_off[u]; j < row_off[u + 1]; ++j) {
            uint32_t a = uf_find(parent, u), b = uf_find(parent, col[j]);
            if (a < b) parent[b] = a; else if (b < a) parent[a] = b;
        }
    for (uint32_t v = 0; v < n; ++v) label[v] = uf_find(parent, v);
    free(parent);
}

/* binary min-heap of (dist, vertex) pairs keyed by dist, lazy deletion */
typedef struct { uint64_t key; uint32_t v; } hent;
static void heap_push(hent* h, uint64_t* sz, hent e) {
    uint64_t i = (*sz)++;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (h[p].key <= e.key) break;
        h[i] = h[p]; i = p;
    }
    h[i] = e;
}
static hent heap_pop(hent* h, uint64_t* sz) {
    hent top = h[0], last = h[--(*sz)];
    uint64_t i = 0;
    for (;;) {
        uint64_t c = 2 * i + 1;
        if (c >= *sz) break;
        if (c + 1 < *sz && h[c + 1].key < h[c].key) c++;
        if (last.key <= h[c].key) break;
        h[i] = h[c]; i = c;
    }
    if (*sz) h[i] = last;
    return top;
}

/*
 * SSSP (Evaluation, Applications: Bellman-Ford's fixed point) = shortest path
 * lengths with non-negative integer weights; INF32 when unreachable. Dijkstra
 * with a binary heap, or Dial's bucket queue when every weight is <= 4096
 * (same result, fewer operations). Distances are accumulated in 64 bits and
 * must fit in 32.
 */
int or_sssp_dist(uint32_t n, const uint64_t* row_off, const uint32_t* col, const uint32_t* w,
                 uint32_t src, uint32_t* dist) {
    uint64_t m = row_off[n];
    uint32_t wmax = 0;
    for (uint64_t j = 0; j < m; ++j) if (w[j] > wmax) wmax = w[j];
    uint64_t* d = (uint64_t*)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
    for (uint32_t v = 0; v < n; ++v) d[v] = UINT64_MAX;
    int rc = 0;
    if (src < n) {
        d[src] = 0;
        if (wmax <= 4096) {
            /* Dial: circular array of wmax+1 buckets, each a singly linked list */
            uint32_t nb = wmax + 1;
            int64_t* bhead = (int64_t*)malloc(nb * sizeof(int64_t));
            for (uint32_t b = 0; b < nb; ++b) bhead[b] = -1;
            /* entries allocated in a growing pool: (vertex, dist, next) */
            uint64_t cap = (uint64_t)n + m + 1, used = 0;
            uint32_t* ev = (uint32_t*)malloc(cap * sizeof(uint32_t));
            uint64_t* ed = (uint64_t*)malloc(cap * sizeof(uint64_t));
            int64_t* en = (int64_t*)malloc(cap * sizeof(int64_t));
            uint64_t pending = 0;
            ev[used] = src; ed[used] = 0; en[used] = bhead[0]; bhead[0] = (int64_t)used++; pending++;
            for (uint64_t cur = 0; pending > 0; ++cur) {
                uint32_t b = (uint32_t)(cur % nb);
                while (bhead[b] >= 0) {
                    int64_t e = bhead[b];
                    bhead[b] = en[e];
                    pending--;
                    uint32_t u = ev[e];
                    if (ed[e] != d[u]) continue;           /* stale entry */
                    for (uint64_t j = row_off[u]; j < row_off[u + 1]; ++j) {
                        uint32_t v = col[j];
                        uint64_t nd = d[u] + w[j];
                        if (nd < d[v]) {
                            d[v] = nd;
                            uint32_t nbk = (uint32_t)(nd % nb);
                            ev[used] = v; ed[used] = nd; en[used] = bhead[nbk];
                            bhead[nbk] = (int64_t)used++; pending++;
                        }
                    }
                }
            }
            free(ev); free(ed); free(en); free(bhead);
        } else {
            hent* h = (hent*)malloc((size_t)(m + 2) * sizeof(hent));
            uint64_t sz = 0;
            hent s0 = {0, src};
            heap_push(h, &sz, s0);
            while (sz) {
                hent t = heap_pop(h, &sz);
                if (t.key != d[t.v]) continue;
                for (uint64_t j = row_off[t.v]; j < row_off[t.v + 1]; ++j) {
                    uint64_t nd = t.key + w[j];
                    if (nd < d[col[j]]) { d[col[j]] = nd; hent e = {nd, col[j]}; heap_push(h, &sz, e); }
                }
            }
            free(h);
        }
    }
    for (uint32_t v = 0; v < n; ++v) {
        if (d[v] == UINT64_MAX) dist[v] = INF32;
        else if (d[v] >= INF32) { dist[v] = INF32; rc = -1; }
        else dist[v] = (uint32_t)d[v];
    }
    free(d);
    return rc;
}

/* Neumaier's compensated summation (Neumaier 1974) */
typedef struct { double s, c; } ksum;
static inline void ks_add(ksum* k, double x) {
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x; else k->c += (x - t) + k->s;
    k->s = t;
}
static inline double ks_val(const ksum* k) { return k->s + k->c; }

/*
 * PageRank power iteration in FP64. The paper names PageRank but gives no
 * formula (Evaluation, Applications); the standard damped form is used:
 *   r_0(v) = 1/N
 *   D_k    = sum of r_k(u) over vertices with out-degree 0
 *   r_{k+1}(v) = (1-d)/N + d * ( sum_{(u,v) in E} r_k(u)/outdeg(u) + D_k/N ).
 * Per-vertex sums walk the in-edges (CSC built here) with compensation;
 * parallel over destinations, so results do not depend on the thread count.
 * nthreads <= 0 uses the OpenMP default.
 */
void or_pagerank(uint32_t n, const uint64_t* row_off, const uint32_t* col, uint32_t iters,
                 double damping, double* rank, int nthreads) {
    if (n == 0) return;
    uint64_t m = row_off[n];
    uint64_t* col_off = (uint64_t*)malloc(((size_t)n + 1) * sizeof(uint64_t));
    uint32_t* in_src = (uint32_t*)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
    or_csc_from_csr(n, row_off, col, NULL, col_off, in_src, NULL);
    double* contrib = (double*)malloc((size_t)n * sizeof(double));
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    for (uint32_t v = 0; v < n; ++v) rank[v] = 1.0 / (double)n;
    for (uint32_t k = 0; k < iters; ++k) {
        ksum dk = {0, 0};
        for (uint32_t u = 0; u < n; ++u) {
            uint64_t od = row_off[u + 1] - row_off[u];
            if (od == 0) { ks_add(&dk, rank[u]); contrib[u] = 0.0; }
            else contrib[u] = rank[u] / (double)od;
        }
        double dangling = ks_val(&dk);
        double base = (1.0 - damping) / (double)n;
#pragma omp parallel for schedule(dynamic, 4096) num_threads(nthreads)
        for (int64_t v = 0; v < (int64_t)n; ++v) {
            ksum s = {0, 0};
            for (uint64_t p = col_off[v]; p < col_off[v + 1]; ++p) ks_add(&s, contrib[in_src[p]]);
            rank[v] = base + damping * (ks_val(&s) + dangling / (double)n);
        }
    }
    free(contrib); free(in_src); free(col_off);
}

/* ---------------------------------------------------- the method, per step */

/*
 * Wedge Frontier of a vertex frontier (Wedge Frontier; Frontier Transformation,
 * "Frontier Precision"): the set of edge groups, each of `chunk` contiguous
 * positions of the in-edge array named by its starting position, that hold at
 * least one in-edge whose source is in the frontier. Computed by a full scan
 * of the in-edge array, independently of any edge index.
 * bits[g] is set to 1 for every marked group g (bits has ceil(m/chunk) bytes).
 * Returns the number of marked groups.
 */
uint64_t or_wedge_frontier(uint64_t m, const uint32_t* in_src, const uint8_t* frontier,
                           uint32_t chunk, uint8_t* bits) {
    uint64_t groups = (m + chunk - 1) / chunk, marked = 0;
    memset(bits, 0, (size_t)groups);
    for (uint64_t p = 0; p < m; ++p)
        if (frontier[in_src[p]]) bits[p / chunk] = 1;
    for (uint64_t g = 0; g < groups; ++g) marked += bits[g];
    return marked;
}

/* candidate value carried by in-edge (u -> v, weight wt) out of value x = val[u] */
static inline uint32_t candidate(int app, uint32_t k, uint32_t xu, uint32_t wt) {
    if (app == APP_BFS) return k + 1;
    if (app == APP_CC) return xu;
    return xu == INF32 ? INF32 : (uint64_t)xu + wt >= INF32 ? INF32 - 1 : xu + wt;
}

static void init_values(int app, uint32_t n, uint32_t src, uint32_t* val, uint8_t* fr) {
    memset(fr, 0, n);
    for (uint32_t v = 0; v < n; ++v) val[v] = (app == APP_CC) ? v : INF32;
    if (app == APP_CC) { memset(fr, 1, n); }
    else if (src < n) { val[src] = 0; fr[src] = 1; }
}

/*
 * Synchronous pull engine with the Wedge control loop (Wedge Overview; Frontier
 * Transformation; Evaluation, "Frontier Fullness Threshold").
 *
 * Each iteration k:
 *   A_k    = sum of out-degrees over the frontier F_k (the "number of edges
 *            the frontier contains");
 *   mode_k = 1 (build and use the Wedge Frontier) when A_k < thr_edges,
 *            0 (pull over the whole graph without a frontier) otherwise;
 *   K_k    = size of the Wedge Frontier of F_k at group size `chunk`, and the
 *            number of in-edges a pull over it would visit (all m in mode 0);
 *   then every destination pulls over its in-edges from F_k only (the active
 *   subset) and a vertex enters F_{k+1} exactly when its value drops.
 * Values: BFS levels (k+1 for a vertex first reached in iteration k), CC labels
 * (min over active in-neighbours), SSSP distances (min of dist[u]+w).
 * For CC pass the undirected view. thr_edges is the threshold in edges
 * (floor(theta * m)); chunk 0 skips the Wedge Frontier size.
 * Trace arrays (nullable) hold max_iters entries; frontiers (nullable) holds
 * max_iters * n bytes, row k being F_k. Returns the iteration count, or -1 if
 * max_iters was reached with a non-empty frontier.
 */
int64_t or_pull_engine(int app, uint32_t n, const uint64_t* row_off, const uint32_t* col,
                       const uint32_t* w, uint32_t src, uint64_t thr_edges, uint32_t chunk,
                       uint32_t max_iters, uint32_t* val, uint64_t* tr_F, uint64_t* tr_A,
                       uint8_t* tr_mode, uint64_t* tr_K, uint64_t* tr_edges, uint8_t* frontiers,
                       int nthreads) {
    uint64_t m = row_off[n];
    uint64_t* col_off = (uint64_t*)malloc(((size_t)n + 1) * sizeof(uint64_t));
    uint32_t* in_src = (uint32_t*)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
    uint32_t* in_w = (uint32_t*)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
    or_csc_from_csr(n, row_off, col, w, col_off, in_src, w ? in_w : NULL);
    uint8_t* fr = (uint8_t*)malloc((size_t)(n ? n : 1));
    uint8_t* fr_next = (uint8_t*)malloc((size_t)(n ? n : 1));
    uint32_t* next = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    uint64_t groups = chunk ? (m + chunk - 1) / chunk : 0;
    uint8_t* bits = (uint8_t*)malloc((size_t)(groups ? groups : 1));
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    init_values(app, n, src, val, fr);
    int64_t iters = -1;
    for (uint32_t k = 0; k < max_iters; ++k) {
        uint64_t fcount = 0, A = 0;
        for (uint32_t u = 0; u < n; ++u)
            if (fr[u]) { fcount++; A += row_off[u + 1] - row_off[u]; }
        if (fcount == 0) { iters = k; break; }
        int mode = A < thr_edges ? 1 : 0;
        uint64_t K = 0, visited = m;
        if (chunk) {
            K = or_wedge_frontier(m, in_src, fr, chunk, bits);
            if (mode) {
                visited = 0;
                for (uint64_t g = 0; g < groups; ++g)
                    if (bits[g]) {
                        uint64_t end = (g + 1) * chunk < m ? (g + 1) * chunk : m;
                        visited += end - g * chunk;
                    }
            }
        }
        if (tr_F) tr_F[k] = fcount;
        if (tr_A) tr_A[k] = A;
        if (tr_mode) tr_mode[k] = (uint8_t)mode;
        if (tr_K) tr_K[k] = K;
        if (tr_edges) tr_edges[k] = visited;
        if (frontiers) memcpy(frontiers + (size_t)k * n, fr, n);
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nthreads)
        for (int64_t v = 0; v < (int64_t)n; ++v) {
            uint32_t best = val[v];
            if (!(app == APP_BFS && best != INF32)) {
                for (uint64_t p = col_off[v]; p < col_off[v + 1]; ++p) {
                    uint32_t u = in_src[p];
                    if (!fr[u]) continue;                       /* outside the active subset */
                    uint32_t c = candidate(app, k, val[u], w ? in_w[p] : 0);
                    if (c < best) best = c;
                }
            }
            next[v] = best;
            fr_next[v] = best < val[v];
        }
        memcpy(val, next, (size_t)n * sizeof(uint32_t));
        uint8_t* t = fr; fr = fr_next; fr_next = t;
        if (k + 1 == max_iters) {
            uint64_t left = 0;
            for (uint32_t u = 0; u < n; ++u) left += fr[u];
            iters = left ? -1 : (int64_t)max_iters;
        }
    }
    if (max_iters == 0) iters = -1;
    free(bits); free(next); free(fr_next); free(fr); free(in_w); free(in_src); free(col_off);
    return iters;
}

/*
 * Textbook push engine with the same synchronous semantics (Background, Push
 * vs. Pull): every frontier vertex sends its value along its out-edges; each
 * destination keeps the minimum of what it receives and its old value.
 * Returns the iteration count (as or_pull_engine) and the per-iteration
 * frontier sizes.
 */
int64_t or_push_engine(int app, uint32_t n, const uint64_t* row_off, const uint32_t* col,
                       const uint32_t* w, uint32_t src, uint32_t max_iters, uint32_t* val,
                       uint64_t* tr_F) {
    uint8_t* fr = (uint8_t*)malloc((size_t)(n ? n : 1));
    uint32_t* next = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    init_values(app, n, src, val, fr);
    int64_t iters = -1;
    for (uint32_t k = 0; k < max_iters; ++k) {
        uint64_t fcount = 0;
        for (uint32_t u = 0; u < n; ++u) fcount += fr[u];
        if (fcount == 0) { iters = k; break; }
        if (tr_F) tr_F[k] = fcount;
        memcpy(next, val, (size_t)n * sizeof(uint32_t));
        for (uint32_t u = 0; u < n; ++u) {
            if (!fr[u]) continue;
            for (uint64_t j = row_off[u]; j < row_off[u + 1]; ++j) {
                uint32_t v = col[j];
                if (app == APP_BFS && val[v] != INF32) continue;
                uint32_t c = candidate(app, k, val[u], w ? w[j] : 0);
                if (c < next[v]) next[v] = c;
            }
        }
        uint64_t left = 0;
        for (uint32_t v = 0; v < n; ++v) { fr[v] = next[v] < val[v]; left += fr[v]; }
        memcpy(val, next, (size_t)n * sizeof(uint32_t));
        if (k + 1 == max_iters) iters = left ? -1 : (int64_t)max_iters;
    }
    free(next); free(fr);
    return iters;
}

int or_threads(void) { return omp_get_max_threads(); }
