/*
 * wedge.h -- C ABI of the MI355X (gfx950) Wedge-Frontier pull engine.
 *
 * The method is the pull-only frontier optimisation of Grossman & Kozyrakis,
 * "A New Frontier for Pull-Based Graph Processing" (arXiv 1903.07754):
 *   1. the pull engine emits the usual source-oriented vertex frontier
 *      (Wedge Overview; Background, Push vs. Pull);
 *   2. a fullness decision compares the frontier's out-edge count with a
 *      threshold (Frontier Transformation, "Frontier Fullness Threshold");
 *   3. below it, the frontier is translated through an edge index into the
 *      Wedge Frontier, a bitmap over groups of contiguous in-edge positions
 *      (Wedge Frontier; Frontier Transformation, "Frontier Precision";
 *      Implementation, Data Structures);
 *   4. the pull then visits only the marked groups, or the whole in-edge
 *      array when the frontier is too full.
 *
 * Conventions for every entry point
 *   - Plain C types only. Vertex ids, levels, labels, distances and weights are
 *     uint32; edge counts and offsets are uint64 at the ABI and must be < 2^32
 *     (in-edge positions are stored in 32 bits on the device). n < 2^31.
 *   - "dev" pointers are device memory owned by the caller (hipMalloc, or
 *     torch.empty(..., device="cuda")); "host" pointers are ordinary memory.
 *   - Work is issued on the caller's HIP stream; every run returns after the
 *     stream has completed it (runs are synchronous for the caller).
 *   - Errors are status codes; nothing throws across the ABI. All argument
 *     checks happen before any device work. wedge_last_error() gives a
 *     thread-local message for the last failure.
 *   - The library's own calls that are not stream ordered (device allocation
 *     and free, synchronous clears, pinned allocation, event creation) never
 *     overlap its own stream captures in another thread (one process-wide
 *     lock), so concurrent runs cannot invalidate a persistent run's capture.
 *   - A graph handle is immutable after creation; one graph must not be used by
 *     two runs at the same time (its cached workspace is shared). A run on a
 *     busy graph returns WEDGE_ERR_BUSY. Different graphs may run concurrently
 *     from different threads. Persistent runs (WEDGE_RUN_PERSISTENT) need
 *     their whole grid resident, so the library runs them one at a time per
 *     device within a process; a persistent run that shares the device with
 *     another process's persistent kernels may stall until the barrier
 *     deadline and fail.
 *
 * Environment (read by the library; all optional)
 *   WEDGE_MAX_DEVICE_BYTES    cap on the device memory one graph may allocate
 *                             (exceeding it gives WEDGE_ERR_OOM).
 *   WEDGE_BARRIER_TIMEOUT_MS  deadline of every grid-barrier wait in persistent
 *                             launches (default 10000); a wait past it makes
 *                             every block exit and the run return WEDGE_ERR_HIP.
 *   WEDGE_HOST_THREADS        threads of the host-side layout build (else
 *                             OMP_NUM_THREADS, else the hardware count).
 *   WEDGE_SLICED_PULL         "1": build the source-sliced in-edge copy for every
 *                             graph, "0": for none; unset: for graphs of at
 *                             least 2^22 edges (read at graph create).
 *   WEDGE_TUNE_CACHE          path of a text file that keeps the autotuner's
 *                             table across processes (read on first use,
 *                             rewritten after every wedge_tune_bfs).
 */
#ifndef WEDGE_H
#define WEDGE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WEDGE_OK = 0,
    WEDGE_ERR_INVALID_ARG = -1,   /* null pointer, id out of range, bad option value */
    WEDGE_ERR_BAD_GRAPH = -2,     /* offsets not monotone, neighbour id >= n, m >= 2^32 ... */
    WEDGE_ERR_NO_WEIGHTS = -3,    /* SSSP on a graph created without weights */
    WEDGE_ERR_OOM = -4,           /* device or host allocation failed (or the WEDGE_MAX_DEVICE_BYTES cap) */
    WEDGE_ERR_HIP = -5,           /* a HIP runtime call or kernel failed; see wedge_last_error() */
    WEDGE_ERR_UNSUPPORTED = -6,   /* operation not available for this graph (e.g. CC needs WEDGE_SYMMETRIZE) */
    WEDGE_ERR_MODEL = -7,         /* learned-gate model missing, corrupt or of the wrong version */
    WEDGE_ERR_NOT_CONVERGED = -8, /* max_iters reached while the frontier was still non-empty */
    WEDGE_ERR_BUSY = -9           /* the graph is in use by another run */
} wedge_status;

typedef struct wedge_graph_s* wedge_graph_t;

/* ------------------------------------------------------------------ graphs */

/* wedge_graph_create_* flags */
#define WEDGE_INPUT_DEVICE 0x1u /* row_off/col/w are device pointers (else host) */
#define WEDGE_SYMMETRIZE   0x2u /* store the undirected view: each u->v (u != v) also as v->u,
                                   duplicates merged, self-loops dropped; required by wedge_cc;
                                   weights are not accepted with this flag */
#define WEDGE_HOST_ONLY    0x4u /* build and keep the layout in host memory only, touching no
                                   GPU: the handle then serves wedge_graph_info/_layout and can
                                   not run applications (WEDGE_ERR_UNSUPPORTED) */
#define WEDGE_KEEP_IDS     0x8u /* keep the caller's vertex order inside the library (by
                                   default vertices are renumbered by decreasing out-degree,
                                   which packs the most-gathered values into few cache lines;
                                   results are always returned in the caller's ids) */

/*
 * Create a graph from out-edges (CSR, Background, Graph Representation):
 * row_off[n+1] (uint64, row_off[0] = 0, non-decreasing, row_off[n] = m),
 * col[m] (uint32 destinations < n), w[m] (uint32 weights, nullable; needed by
 * wedge_sssp). Self-loops and duplicate edges are accepted as given (PageRank
 * counts them in the out-degree).
 *
 * The library copies what it needs; the caller may free its arrays on return.
 * It builds, once (the layout of the method's one-off preprocessing):
 *   - the in-edge array (CSC) with each destination's in-edges ordered by
 *     ascending source, weights aligned with it;
 *   - the edge index (Wedge Frontier; Implementation, Data Structures): for
 *     every CSR edge u->v, the position of that edge in the in-edge array,
 *     stored in CSR order so a vertex's entries are contiguous;
 *   - an internal vertex order by decreasing out-degree (unless WEDGE_KEEP_IDS),
 *     applied to every array below; inputs (sources, frontiers) and outputs use
 *     the caller's ids;
 *   - per 64-position row of the in-edge array, a 64-bit mask of the positions
 *     where a destination's in-edge list begins, the index of the destination
 *     segment covering the row's first position, and the list of destinations
 *     with at least one in-edge. These name each position's destination
 *     without the vertex index (the role the paper gives Vector-Sparse);
 *   - for large graphs (see WEDGE_SLICED_PULL), a second copy of the in-edges
 *     split into 8 slices by source (groups of 1024 consecutive internal
 *     ids dealt to the slices in turn), each grouped by destination with its
 *     own row layout. The CC and SSSP pulls over every in-edge run slice j on
 *     the 8th of the GPU's workgroups that the hardware places on XCD j, so
 *     each XCD's L2 caches only its slice's source values.
 * The stream orders the uploads; the call returns after they finish.
 * Returns WEDGE_ERR_BAD_GRAPH for malformed input, WEDGE_ERR_OOM on allocation
 * failure. *out is set only on success.
 */
wedge_status wedge_graph_create_csr(uint32_t n, uint64_t m, const uint64_t* row_off,
                                    const uint32_t* col, const uint32_t* w, uint32_t flags,
                                    hipStream_t stream, wedge_graph_t* out);

/* Same, from in-edges: col_off[n+1], src[m] (sources of each destination's
 * in-edges), w[m] aligned with src. */
wedge_status wedge_graph_create_csc(uint32_t n, uint64_t m, const uint64_t* col_off,
                                    const uint32_t* src, const uint32_t* w, uint32_t flags,
                                    hipStream_t stream, wedge_graph_t* out);

/* Frees device and host memory of the graph. Null is accepted. */
wedge_status wedge_graph_destroy(wedge_graph_t g);

typedef struct {
    uint32_t n;            /* vertices */
    uint64_t m;            /* stored directed edges (after WEDGE_SYMMETRIZE, both directions) */
    uint32_t nonempty;     /* destinations with at least one in-edge */
    uint64_t rows;         /* ceil(m / 64) */
    uint32_t flags;        /* creation flags */
    uint32_t weighted;     /* 1 when weights are stored */
    uint32_t dangling;     /* vertices with out-degree 0 */
    uint32_t pr_tile_edges;/* in-edges per PageRank pull tile */
    uint64_t pr_spans;     /* destinations whose in-edges cross a PageRank tile boundary */
    uint64_t device_bytes; /* device memory held by the graph (layout + cached workspace) */
    uint64_t pr_short_spans; /* of pr_spans, those over at most 9 tiles (listed first) */
    uint32_t relabeled;    /* 1 when the internal vertex order differs from the caller's */
    uint64_t xs_rows;      /* rows of the source-sliced in-edge copy (0: not built) */
    uint64_t xs_segments;  /* its destination segments */
    uint64_t xs_pr_spans;  /* destinations with a sliced-copy segment that crosses a
                              PageRank tile boundary (short ones listed first) */
    uint64_t xs_pr_short_spans; /* of xs_pr_spans, those whose crossing segments
                                   cover at most 8 extra tiles in all */
    uint64_t xs_pr_span_pairs;  /* crossing segments over all of them */
    uint32_t xs_packed;    /* 1: each sliced-copy word is (slice-local source << 8) | weight
                              (weighted graphs with weights <= 255 and n <= 2^27) */
    uint32_t xs_slices;    /* source slices S of the sliced copy (a power of two, 8..64; 0: none) */
} wedge_graph_info;

wedge_status wedge_graph_get_info(wedge_graph_t g, wedge_graph_info* info);

/* Layout arrays that wedge_graph_layout can copy out (for inspection and tests). */
typedef enum {
    WEDGE_LAYOUT_COL_OFF = 0, /* uint32[n+1] in-edge offsets */
    WEDGE_LAYOUT_IN_SRC = 1,  /* uint32[m] source of each in-edge position */
    WEDGE_LAYOUT_IN_W = 2,    /* uint32[m] weight of each in-edge position */
    WEDGE_LAYOUT_ROW_OFF = 3, /* uint32[n+1] out-edge offsets */
    WEDGE_LAYOUT_POS = 4,     /* uint32[m] edge index: in-edge position of each CSR edge */
    WEDGE_LAYOUT_ROWMASK = 5, /* uint64[rows] segment-start bits per 64 positions */
    WEDGE_LAYOUT_ROWSEG = 6,  /* uint32[rows] segment index covering the row's first position */
    WEDGE_LAYOUT_NZDST = 7,   /* uint32[nonempty] destination of each segment */
    WEDGE_LAYOUT_PR_SPANS = 8,/* uint32[3*pr_spans] (vertex, first tile, last tile) */
    WEDGE_LAYOUT_PERM = 9,    /* uint32[n] internal id of each caller id (relabelled graphs) */
    /* the source-sliced copy of the in-edges (graphs with xs_rows > 0): */
    WEDGE_LAYOUT_XS_SRC = 10,     /* uint32[64*xs_rows] sources, or packed words when
                                     xs_packed (the slice-local id i of slice j's source is
                                     its index among the ids of the slice's 1024-id groups,
                                     groups dealt to the S slices in the order 0..S-1, S-1..0, ...);
                                     padding positions hold 0 */
    WEDGE_LAYOUT_XS_W = 11,       /* uint32[64*xs_rows] weights (weighted, not packed) */
    WEDGE_LAYOUT_XS_ROWMASK = 12, /* uint64[xs_rows] */
    WEDGE_LAYOUT_XS_ROWSEG = 13,  /* uint32[xs_rows] */
    WEDGE_LAYOUT_XS_NZDST = 14,   /* uint32[xs_segments] */
    WEDGE_LAYOUT_XS_BOUNDS = 15,  /* uint32[2*S+1]: first row of slices 0..S, then the end
                                     position of slices 0..S-1 (S = xs_slices) */
    /* PageRank fix-up lists of the sliced copy (empty when xs_pr_spans is 0): */
    WEDGE_LAYOUT_XS_PR_SPAN_V = 16,     /* uint32[xs_pr_spans] destination */
    WEDGE_LAYOUT_XS_PR_SPAN_OFF = 17,   /* uint32[xs_pr_spans+1] first pair of each */
    WEDGE_LAYOUT_XS_PR_SPAN_TILES = 18  /* uint32[2*xs_pr_span_pairs] (first tile, last tile)
                                           of each crossing segment, in slice order */
} wedge_layout_array;

/* Layout arrays are indexed and valued by internal vertex ids. */

/* Copy one layout array into host memory `dst` of `bytes` bytes (must be exactly
 * the array's size). Synchronous. */
wedge_status wedge_graph_layout(wedge_graph_t g, wedge_layout_array which, void* dst,
                                uint64_t bytes);

/* ------------------------------------------------------------ applications */

typedef enum {
    WEDGE_GATE_THRESHOLD = 0,    /* Wedge Frontier iff A_k < floor(theta * m) (the paper's rule) */
    WEDGE_GATE_ALWAYS_WEDGE = 1, /* build the Wedge Frontier every iteration */
    WEDGE_GATE_ALWAYS_FULL = 2,  /* never build it: pull over all in-edges every iteration */
    WEDGE_GATE_LEARNED = 3,      /* learned cost model (see wedge_model_*); falls back to the
                                    threshold rule when no valid model is given */
    WEDGE_GATE_ALWAYS_PUSH = 4,  /* baseline: the push engine every iteration (Background, Push
                                    vs. Pull): each frontier vertex sends its value along its
                                    out-edges, destinations updated by atomics */
    WEDGE_GATE_HYBRID = 5        /* baseline: the hybrid engine the paper compares against
                                    (Background, Hybrid Graph Processing): push iff
                                    A_k < floor(theta * m), else a pull over every in-edge; theta
                                    defaults to 5% (threshold_ppm 0 = 50000) for every application */
} wedge_gate;

/* per-iteration record written to wedge_opts.trace */
typedef struct {
    uint32_t iter;          /* k */
    uint32_t mode;          /* 0 = full pull, 1 = Wedge Frontier, 2 = push */
    uint32_t chunk_edges;   /* group size used (mode 1) */
    uint32_t reserved;
    uint64_t frontier;      /* |F_k| */
    uint64_t active_edges;  /* A_k = sum of out-degrees over F_k */
    uint64_t marked_chunks; /* K_k = marked groups (mode 1; 0 in mode 0) */
    float ms;               /* device time of the iteration (WEDGE_RUN_TIME_ITERS) */
    float reserved2;
} wedge_iter_record;

/* wedge_opts.flags */
#define WEDGE_RUN_TIME_PULL  0x1u /* HIP events around each pull launch; sums into stats */
#define WEDGE_RUN_TIME_ITERS 0x2u /* HIP events around each iteration; into trace[k].ms */
#define WEDGE_RUN_PERSISTENT 0x4u /* BFS kinds only: run the whole traversal as one persistent
                                     kernel (grid barriers between steps, the fullness gate
                                     evaluated on the device), captured once in a hipGraph and
                                     replayed; per-iteration times are not available */
#define WEDGE_RUN_INPLACE    0x8u /* CC and SSSP pull gates only: the pull reads sources' values
                                     as this iteration lowers them (asynchronous, Gauss-Seidel
                                     style) instead of the values committed at the end of the
                                     previous iteration, so a drop can travel several hops in one
                                     iteration (the multi-hop propagation the paper observes
                                     with coarse groups; Evaluation, Frontier Precision). The
                                     result is the same fixed point, bit for bit, in at most as
                                     many iterations; the per-iteration frontiers then depend on
                                     the schedule. WEDGE_ERR_UNSUPPORTED for BFS kinds, PageRank
                                     and the push and hybrid gates */

typedef struct {
    uint32_t gate;           /* wedge_gate */
    uint32_t threshold_ppm;  /* theta in parts per million of the traversed edge count; 0 = the
                                application default (BFS 10000 = 1%, CC 200000 = 20%,
                                SSSP 50000 = 5%; the hybrid gate: 50000 = 5%) */
    uint32_t chunk_edges;    /* edges per Wedge Frontier bit: a power of two in [1, 4096];
                                0 = application default (BFS 32, CC/SSSP 16) */
    uint32_t max_iters;      /* 0 = unlimited (n + 1 bounds every application) */
    uint32_t flags;          /* WEDGE_RUN_* */
    uint32_t trace_cap;      /* entries available at trace */
    wedge_iter_record* trace;/* host array, nullable */
    const void* model;       /* wedge_model_t for WEDGE_GATE_LEARNED, nullable */
    uint32_t blocks_per_cu;  /* WEDGE_RUN_PERSISTENT: resident blocks per compute unit (blocks
                                of 512 threads for multi-source BFS, 768 otherwise); 0 = as many
                                as the kernel's occupancy allows (the value is clamped to that
                                maximum so every block is co-resident) */
    uint32_t rows_per_wave;  /* host-driven BFS, multi-source and batch runs: 64-edge rows a
                                wave pulls per step, 4, 8 or 16 (0 = 8); results do not
                                depend on it. Other runs take 0 or 8 */
} wedge_opts;

typedef struct {
    uint32_t iterations;     /* pull iterations executed */
    uint32_t wedge_iters;    /* of which used the Wedge Frontier */
    uint32_t full_iters;     /* of which pulled over every in-edge */
    uint32_t pull_launches;  /* pull kernel launches (timed when WEDGE_RUN_TIME_PULL) */
    uint64_t edges_scanned;  /* in-edge positions the pull kernels covered */
    double ms;               /* host wall time of the run, sync to sync */
    double pull_ms;          /* sum of event-timed pull kernel durations */
    double full_pull_ms;     /* of which the pulls over every in-edge */
    uint32_t full_pull_launches; /* timed pulls over every in-edge */
    uint32_t push_iters;     /* iterations run by the push engine (push and hybrid gates) */
} wedge_stats;

/*
 * BFS (Evaluation, Applications): level_dev[n] receives the hop level of every
 * vertex from src, 0xFFFFFFFF when unreachable. opts and stats are nullable.
 *
 * BFS, CC and SSSP share one iteration semantics whatever engine runs an
 * iteration (the Wedge pull, the pull over every in-edge, or the push
 * engine of the baseline gates): iteration k uses the values committed at
 * the end of iteration k-1, and a vertex joins the next frontier exactly when
 * its value drops. Results and per-iteration frontiers are therefore the same
 * under every gate. The push engine needs the graph's out-edges in CSR order;
 * the first push or hybrid run on a graph builds them on the device (4 bytes
 * per edge, 8 with weights) and keeps them with the graph.
 */
wedge_status wedge_bfs(wedge_graph_t g, uint32_t src, uint32_t* level_dev, const wedge_opts* opts,
                       hipStream_t stream, wedge_stats* stats);

/*
 * BFS that allocates nothing: for callers that cannot allocate device or
 * pinned memory during the run (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc). Same arguments, results and
 * per-iteration trace as wedge_bfs, from the same kernels; the graph (made
 * beforehand) and level_dev (the caller's) are the only other memory used.
 * The workspace lives in a fixed device array of 32 MiB that the library
 * holds on each GPU it runs on until the process ends (looked up once per
 * device, on its first call there). It needs, in bytes, rounded up to 256
 * each: 64 (counters) + 2 * ceil(n/64) * 8 (frontier bitmaps) + 8n (frontier
 * list and out-degree prefix) + 4n (values, unless created with
 * WEDGE_KEEP_IDS) + ceil(ceil(m/C)/64) * 8 + ceil(m/C) * 4 (Wedge bitmap and
 * marked-group list), C = chunk_edges (default 32); a graph needing more is
 * refused with WEDGE_ERR_INVALID_ARG before any device work (about n = 2.4M
 * at 16 edges per vertex). The graph's device must be current
 * (WEDGE_ERR_INVALID_ARG otherwise). Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents (each call clears what must
 * start at zero): calls that overlapped on one GPU would race, so the library
 * runs them one at a time per device within a process. Refused with
 * WEDGE_ERR_UNSUPPORTED: WEDGE_GATE_LEARNED (its model buffers are
 * allocated on first use), the push and hybrid gates (their out-edge arrays
 * are built on first use) and any wedge_opts.flags bit (timing events,
 * persistent launch buffers).
 */
wedge_status wedge_bfs_noalloc(wedge_graph_t g, uint32_t src, uint32_t* level_dev,
                               const wedge_opts* opts, hipStream_t stream, wedge_stats* stats);

/*
 * Connected components by label propagation (HCC; Evaluation, Applications)
 * on an undirected graph (created with WEDGE_SYMMETRIZE): label_dev[n]
 * receives the smallest vertex id of each component.
 */
wedge_status wedge_cc(wedge_graph_t g, uint32_t* label_dev, const wedge_opts* opts,
                      hipStream_t stream, wedge_stats* stats);

/*
 * Single-source shortest paths by Bellman-Ford (Evaluation, Applications):
 * dist_dev[n] receives path lengths with the stored uint32 weights,
 * 0xFFFFFFFF when unreachable. Requires weights (WEDGE_ERR_NO_WEIGHTS) and
 * (n-1) * max weight < 2^32 - 1 (WEDGE_ERR_INVALID_ARG otherwise).
 */
wedge_status wedge_sssp(wedge_graph_t g, uint32_t src, uint32_t* dist_dev, const wedge_opts* opts,
                        hipStream_t stream, wedge_stats* stats);

/*
 * PageRank (named by the paper, which excludes it from the frontier study as it
 * has no frontier; Evaluation, Applications): `iters` full pulls of
 *   r_{k+1}(v) = (1-d)/n + d * (sum_{u->v} r_k(u)/outdeg(u) + D_k/n),
 * r_0 = 1/n, D_k = rank mass on out-degree-0 vertices. rank_dev[n] (FP32)
 * receives r_iters. 0 < damping < 1. Results are deterministic (no float
 * atomics). The gate and chunk options are ignored.
 */
wedge_status wedge_pagerank(wedge_graph_t g, uint32_t iters, float damping, float* rank_dev,
                            const wedge_opts* opts, hipStream_t stream, wedge_stats* stats);

/* ---------------------------------------------------------- learned gate */

/*
 * A small learned cost model for the fullness decision: an FP32 MLP
 * 8 -> 32 -> 32 -> 4 (ReLU) predicting, for each mode, log(1 + microseconds)
 * of the next iteration minus that of the full pull (mode 0 = full pull,
 * modes 1, 2, 3 = Wedge Frontier at 16, 32, 64 edges per bit); a model is an
 * ensemble of such MLPs and predicts their mean. With WEDGE_GATE_LEARNED the
 * decision is computed on the device between iterations: the mode of
 * smallest prediction (ties to the lower index) when it is predicted faster
 * than the threshold rule's mode by more than the model's decision margin
 * (wedge_model_margin), else the threshold rule's mode. The paper's
 * threshold rule (Frontier Transformation, Frontier Fullness Threshold) also
 * decides when no model is given or a feature lies outside the model's
 * training envelope. The choice never changes results (any mode visits a
 * superset of the active edges).
 *
 * Features of the frontier F_k about to be consumed (float, in this order):
 * |F_k|/n, A_k/m, 1 - exp(-A_k/ceil(m/16)), WEDGE_APP_* / 3, log2(m)/32,
 * min(k,255)/64, log(1 + previous iteration's device time in us)/16,
 * previous mode index / 3.
 */
typedef struct wedge_model_s* wedge_model_t;

#define WEDGE_APP_BFS 1u
#define WEDGE_APP_CC 2u
#define WEDGE_APP_SSSP 3u

/* One iteration of a counterfactual trace (what the model learns from). */
typedef struct {
    uint32_t app;            /* WEDGE_APP_* */
    uint32_t iter;           /* k */
    uint32_t prev_mode;      /* mode index taken at k-1 by the threshold rule (0 at k = 0) */
    uint32_t threshold_mode; /* mode index the threshold rule takes at k */
    uint64_t n, m;           /* traversed graph size */
    uint64_t frontier;       /* |F_k| */
    uint64_t active;         /* A_k */
    float prev_us;           /* device time of iteration k-1 in prev_mode (0 at k = 0) */
    float t_us[4];           /* device time of iteration k in each mode, all from the same state */
    float reserved;
} wedge_trace_sample;

/* New model with uniform(+-1/sqrt(fan_in)) weights from `seed`, zero biases,
 * and an unbounded envelope. Host-only until first used on a GPU. */
wedge_status wedge_model_create(uint64_t seed, wedge_model_t* out);
/* New ensemble of `members` (1..8) such MLPs, drawn one after another from
 * `seed` (member 0 equals wedge_model_create's model). The ensemble predicts
 * the mean of its members' outputs, on the device and in wedge_model_predict;
 * training trains every member on its own. WEDGE_ERR_INVALID_ARG outside 1..8. */
wedge_status wedge_model_create_ensemble(uint64_t seed, uint32_t members, wedge_model_t* out);
/* Number of ensemble members of m. */
wedge_status wedge_model_members(wedge_model_t m, uint32_t* members);
wedge_status wedge_model_free(wedge_model_t m);
/* Versioned binary file: magic "WEDGEMLP", version, shape, member count,
 * decision margin, envelope, 1476 parameters per member, FNV-1a-64 checksum
 * (version 4; version 3 files without the margin and version 2 files with
 * one MLP still load, with margin 0). Load returns WEDGE_ERR_MODEL for a
 * missing, truncated, corrupt or mismatched file. */
wedge_status wedge_model_load(const char* path, wedge_model_t* out);
wedge_status wedge_model_save(wedge_model_t m, const char* path);
/* Copy the 1476 x members parameters (per member W1[32x8] b1 W2[32x32] b2
 * W3[4x32] b3, row-major; members one after another) out (set = 0) or in
 * (set = 1); count must equal 1476 x members. */
wedge_status wedge_model_params(wedge_model_t m, float* params, uint32_t count, int set);
/* Decision margin (>= 0, default 0), read (set = 0) or written (set = 1).
 * Inside the envelope the learned gate takes the model's choice (the argmin
 * of the members' mean predicted log-times) only when its predicted time is
 * below that of the threshold rule's choice by more than the margin;
 * otherwise it keeps the threshold rule's decision. 0 = the plain argmin.
 * WEDGE_ERR_INVALID_ARG for a negative or non-finite margin. */
wedge_status wedge_model_margin(wedge_model_t m, float* margin, int set);
/* Copy the per-feature envelope lo[8], hi[8] out (set = 0) or in (set = 1). */
wedge_status wedge_model_envelope(wedge_model_t m, float* lo, float* hi, int set);
/* Features of samples (host): x[count*8]. */
wedge_status wedge_model_features(const wedge_trace_sample* s, uint32_t count, float* x);
/* y[count*4] = model(x[count*8]) on the device (host arrays). */
wedge_status wedge_model_predict(wedge_model_t m, const float* x, uint32_t count, float* y,
                                 hipStream_t stream);
/* Gradient of mean_b sum_j mask[b,j] (y[b,j] - t[b,j])^2 with respect to the
 * parameters, and the loss, on the device (host arrays). One-member models
 * only (WEDGE_ERR_UNSUPPORTED otherwise). */
wedge_status wedge_model_grad(wedge_model_t m, const float* x, const float* t, const float* mask,
                              uint32_t count, float* grad, float* loss, hipStream_t stream);
/* Full-batch Adam (lr, 0.9, 0.999, 1e-8) on log(1 + t_us[j]) - log(1 + t_us[0])
 * targets (samples without a full-pull time are ignored) for
 * `epochs` steps on the device, each ensemble member on its own from its own
 * initial parameters (final_loss: the members' mean); sets the envelope to the samples' feature
 * range widened by 5%, except for the graph-size and previous-time features
 * (4, 6), which stay unbounded so that a model trained on small graphs is
 * used on larger ones. */
wedge_status wedge_model_train(wedge_model_t m, const wedge_trace_sample* s, uint32_t count,
                               uint32_t epochs, float lr, hipStream_t stream, float* final_loss);

/*
 * Counterfactual per-iteration trace (the profiling method of the paper's
 * Evaluation, Frontier Fullness Threshold: per-iteration times with and
 * without the Wedge Frontier): the app runs as under the threshold rule, and
 * at every iteration the state is saved, the iteration is run and timed in all
 * four modes from that same state (restoring between runs), and the traversal
 * advances. Writes up to cap samples to out (host) and their number to *count.
 * opts supplies theta and the default chunk size of the threshold rule.
 */
wedge_status wedge_trace_counterfactual(wedge_graph_t g, uint32_t app, uint32_t src,
                                        const wedge_opts* opts, wedge_trace_sample* out,
                                        uint32_t cap, uint32_t* count, hipStream_t stream);

/* ------------------------------------------------------------- batching */

/*
 * Multi-source BFS: `count` (1..64) BFS runs from srcs[0..count) (host array of
 * caller ids) in one traversal, each vertex holding a 64-bit mask per state
 * (bit s = source s), after Then et al., "The More the Merrier" (PVLDB 8(4),
 * 2014). The Wedge machinery runs on the union frontier {v : some source
 * reached v in the last iteration} with the usual gate and chunk options.
 * levels_dev[s*n + v] receives the level of v from srcs[s] (0xFFFFFFFF when
 * unreachable); the caller provides count*n entries.
 */
wedge_status wedge_bfs_multisource(wedge_graph_t g, const uint32_t* srcs, uint32_t count,
                                   uint32_t* levels_dev, const wedge_opts* opts,
                                   hipStream_t stream, wedge_stats* stats);

/*
 * One graph holding `count` independent graphs as a disjoint union: part i has
 * n_each[i] vertices and out-edges row_off[i], col[i] (host arrays, part-local
 * ids), and becomes vertices [first_i, first_i + n_each[i]) of the union.
 * Flags as for wedge_graph_create_csr (weights are not supported).
 */
wedge_status wedge_graph_create_batch_csr(uint32_t count, const uint32_t* n_each,
                                          const uint64_t* const* row_off,
                                          const uint32_t* const* col, uint32_t flags,
                                          hipStream_t stream, wedge_graph_t* out);

/* First vertex of each part of a batch graph: first[0..count] (first[count] = n). */
wedge_status wedge_graph_batch_parts(wedge_graph_t g, uint64_t* first, uint32_t cap,
                                     uint32_t* count);

/*
 * One BFS per part of a batch graph in a single traversal: srcs[i] (host) is
 * the part-local source of part i. The union is traversed from all sources at
 * once; parts share no edges, so each vertex gets its own part's level.
 * levels_dev[n] receives the levels in union order.
 */
wedge_status wedge_bfs_batch(wedge_graph_t g, const uint32_t* srcs, uint32_t* levels_dev,
                             const wedge_opts* opts, hipStream_t stream, wedge_stats* stats);

/* kinds for wedge_tune_bfs */
#define WEDGE_TUNE_SINGLE 0u      /* wedge_bfs from srcs[0] */
#define WEDGE_TUNE_MULTISOURCE 1u /* wedge_bfs_multisource over srcs[0..count) */
#define WEDGE_TUNE_BATCH 2u       /* wedge_bfs_batch with srcs[0..parts) */

/*
 * Autotuner: times the BFS kind on this graph and these sources for every
 * combination of edges per Wedge bit {16, 32, 64} with, for the host-driven
 * loop, rows per wave {4, 8, 16} and, for the persistent launch, blocks per
 * compute unit (1, 2 and 4 where below the occupancy maximum, and that
 * maximum); best of two runs each. It writes the fastest options to *best (its gate
 * and threshold are taken from *best on entry). Results do not depend on the
 * choice. out_dev is scratch output of the kind's size. The winner is also
 * kept in a process-wide table keyed by (kind, source count, ceil(log2 m),
 * the device's compute unit count), which wedge_tune_lookup reads, and, when
 * WEDGE_TUNE_CACHE names a file, in that file, so later processes find it.
 */
wedge_status wedge_tune_bfs(wedge_graph_t g, uint32_t kind, const uint32_t* srcs, uint32_t count,
                            uint32_t* out_dev, hipStream_t stream, wedge_opts* best,
                            double* best_ms);

/* Tuned options for (kind, count, edge count m) on the current device, if
 * wedge_tune_bfs has recorded them in this process or in the WEDGE_TUNE_CACHE
 * file: copies chunk_edges, flags' persistent bit, blocks_per_cu and
 * rows_per_wave into *opts and returns WEDGE_OK; else WEDGE_ERR_UNSUPPORTED. */
wedge_status wedge_tune_lookup(uint32_t kind, uint32_t count, uint64_t m, wedge_opts* opts);

/* ------------------------------------------------------- single steps */

/*
 * Frontier transformation alone (Wedge Frontier; Implementation, Data
 * Structures): for the vertex frontier frontier_dev[count] (distinct vertex
 * ids, any order), set bit g of wbits_dev for every group g of chunk_edges
 * in-edge positions holding an out-edge of a frontier vertex, then compact the
 * bitmap into chunk_list_dev (marked group ids, any order) and return their
 * number in *marked. wbits_dev has ceil(ceil(m/chunk_edges)/64) uint64 words
 * and is overwritten; chunk_list_dev holds ceil(m/chunk_edges) entries.
 */
wedge_status wedge_frontier_translate(wedge_graph_t g, const uint32_t* frontier_dev,
                                      uint32_t count, uint32_t chunk_edges, uint64_t* wbits_dev,
                                      uint32_t* chunk_list_dev, uint64_t* marked,
                                      hipStream_t stream);

/* ------------------------------------------------------------------ misc */

const char* wedge_status_string(wedge_status s);
const char* wedge_last_error(void);
/* Library version, e.g. "0.1.0". */
const char* wedge_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WEDGE_H */
