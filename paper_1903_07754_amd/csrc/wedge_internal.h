// Internal declarations shared by the host driver (api.cpp, layout.cpp) and the
// HIP kernels (kernels.hip). Not part of the public ABI.
#pragma once

#include <stdint.h>
#include <stddef.h>

#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/wedge.h"

namespace wedge {

constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr int kWave = 64;
constexpr int kPullRows = 8;         // default rows (64 positions each) per wave in the integer pulls
constexpr uint32_t kPrTileRows = 8;  // PageRank pull tile: 8 rows of 64 in-edge positions
constexpr uint32_t kPrShortSpan = 8; // spans over at most this many extra tiles are fixed up per lane
constexpr int kMaxSlices = 64;       // most source slices of the sliced full pulls
constexpr int kXcdGroupShift = 10;   // source slices deal out groups of 1024 vertices

enum App : int { kBfs = 1, kCc = 2, kSssp = 3 };

// ------------------------------------------------------------- host layout
// Everything the device needs, built once on the host from the input graph.
struct HostLayout {
    uint32_t n = 0;
    uint64_t m = 0;
    std::vector<uint32_t> col_off;   // n+1
    std::vector<uint32_t> in_src;    // m
    std::vector<uint32_t> in_w;      // m (empty when unweighted)
    std::vector<uint32_t> row_off;   // n+1
    std::vector<uint32_t> pos;       // m, CSR order
    std::vector<uint64_t> rowmask;   // rows
    std::vector<uint32_t> rowseg;    // rows
    std::vector<uint32_t> nzdst;     // nonempty
    std::vector<uint32_t> spans;     // 3 * pr_spans (v, first tile, last tile); short ones first
    uint64_t short_spans = 0;
    std::vector<uint32_t> perm;      // original id -> internal id (empty: identity)
    std::vector<uint32_t> inv;       // internal id -> original id
    uint32_t dangling = 0;
    uint32_t max_w = 0;
    // source-sliced copy of the in-edges for the CC/SSSP full pulls (empty
    // when not built): slice j holds the in-edges whose source lies in slice
    // j (xcd_slice_of), grouped by destination like the canonical array, and
    // starts at row xs_row_begin[j]; positions from xs_edge_end[j] to the
    // next slice's first row are padding
    std::vector<uint32_t> xs_src, xs_w, xs_rowseg, xs_nzdst;
    std::vector<uint64_t> xs_rowmask;
    // packed form (weighted graphs with weights <= 255 and n <= 2^27): xs_src
    // holds (slice-local source << 8) | weight and xs_w is empty
    bool xs_packed = false;
    // PageRank over the sliced copy: destinations with segments crossing a
    // tile boundary (short ones first), the offsets of their (first tile,
    // last tile) pairs, and the pairs
    std::vector<uint32_t> xs_pspan_v, xs_pspan_off, xs_pspan_tt;
    uint64_t xs_pspan_short = 0;
    uint32_t xs_lg = 0;  // log2 of the number of slices
    uint32_t xs_row_begin[kMaxSlices + 1] = {};
    uint32_t xs_edge_end[kMaxSlices] = {};
};

// Source slice of internal vertex u for the sliced full pulls, with 2^lg
// slices: 1024-vertex groups (4 KB of 32-bit values, whole cache lines) dealt
// to the slices in a snake order (0..S-1, S-1..0, ...), which balances the
// out-degree-sorted vertices' edges across slices. The slices are pulled one
// launch after another, so at any time the L2 of every XCD only needs the
// values of one slice's sources (1/S of the array).
__host__ __device__ inline uint32_t xcd_slice_of(uint32_t u, uint32_t lg) {
    const uint32_t g = u >> kXcdGroupShift;
    const uint32_t r = g & ((1u << lg) - 1u);
    return ((g >> lg) & 1u) ? (1u << lg) - 1u - r : r;
}
// Index of u among its slice's vertices (the slice's groups in order), and
// back: the slice-local ids of a slice's highest-out-degree sources are the
// lowest.
__host__ __device__ inline uint32_t xcd_slice_local(uint32_t u, uint32_t lg) {
    return ((u >> (kXcdGroupShift + lg)) << kXcdGroupShift) | (u & ((1u << kXcdGroupShift) - 1u));
}
__host__ __device__ inline uint32_t xcd_slice_global(uint32_t i, uint32_t j, uint32_t lg) {
    const uint32_t b = i >> kXcdGroupShift;
    const uint32_t gidx = (b << lg) + ((b & 1u) ? (1u << lg) - 1u - j : j);
    return (gidx << kXcdGroupShift) | (i & ((1u << kXcdGroupShift) - 1u));
}
// The number of slices for a graph with `sources` vertices that have
// out-edges (the values a full pull gathers): the smallest power of two from
// 8 to kMaxSlices whose slices hold at most kSliceValueBytes of their 32-bit
// values, twice an XCD's L2 (WEDGE_XS_SLICES overrides it). Measured at
// scale 24 and 26: 8 slices for R-MAT s24 (7.4M sources), 16 for ER s24
// (16.8M) and for R-MAT s26 (27.1M); more slices cost more than they save
// (each destination's value is read once per slice it has in-edges in).
constexpr uint64_t kSliceValueBytes = 8ull << 20;
uint32_t xs_slices_lg(uint64_t sources);
// The packed sliced copy: (slice-local source << 8) | weight in one word.
constexpr uint32_t kXsPackMaxW = 255;
// Rows of padding after the row layout's masks and segment indices on the
// device (mask 1, the last segment index): the full pulls read the entries of
// a wave's rows and the row after them without clamping to the layout.
constexpr uint32_t kRowPad = 32;
constexpr uint64_t kXsPackMaxN = 1ull << 27;  // slice-local ids below 2^24 (at least 8 slices)

// Builds the source-sliced copy of L's in-edges (L must hold the canonical layout).
void build_xcd_slices(HostLayout* L);

// Validates and builds the layout from CSR (edges grouped by source) or CSC
// (grouped by destination). Returns WEDGE_OK or an error with *err set.
wedge_status build_layout_from_csr(uint32_t n, uint64_t m, const uint64_t* row_off,
                                   const uint32_t* col, const uint32_t* w, bool symmetrize,
                                   bool relabel, HostLayout* out, std::string* err);
wedge_status build_layout_from_csc(uint32_t n, uint64_t m, const uint64_t* col_off,
                                   const uint32_t* src, const uint32_t* w, bool symmetrize,
                                   bool relabel, HostLayout* out, std::string* err);

// ------------------------------------------------------- device structures
struct DevGraph {
    uint32_t n = 0;
    uint64_t m = 0;
    uint64_t rows = 0;
    uint32_t nonempty = 0;
    uint64_t nspans = 0;
    uint64_t short_spans = 0;
    uint32_t* col_off = nullptr;
    uint32_t* in_src = nullptr;
    uint32_t* in_w = nullptr;
    uint32_t* row_off = nullptr;
    uint32_t* pos = nullptr;
    uint64_t* rowmask = nullptr;
    uint32_t* rowseg = nullptr;
    uint32_t* nzdst = nullptr;
    uint32_t* spans = nullptr;
    uint32_t* perm = nullptr;  // original -> internal (null: identity)
    uint32_t* inv = nullptr;   // internal -> original (null: identity)
    // source-sliced in-edges for the CC/SSSP full pulls (null: not built)
    uint32_t* xs_src = nullptr;
    uint32_t* xs_w = nullptr;
    uint64_t* xs_rowmask = nullptr;
    uint32_t* xs_rowseg = nullptr;
    uint32_t* xs_nzdst = nullptr;
    uint64_t xs_rows = 0;
    bool xs_packed = false;     // xs_src holds (slice-local source << 8) | weight
    int cus = 0;                // compute units of the graph's device
    uint64_t xs_positions = 0;  // padded length
    uint64_t xs_segments = 0;
    uint32_t* xs_pspan_v = nullptr;
    uint32_t* xs_pspan_off = nullptr;
    uint32_t* xs_pspan_tt = nullptr;
    uint64_t xs_pspans = 0;       // destinations with crossing segments
    uint64_t xs_pspan_short = 0;  // of which listed first as short
    uint64_t xs_pspan_pairs = 0;  // crossing segments over all of them
    uint32_t xs_lg = 0;         // log2 of the number of slices
    uint32_t xs_row_begin[kMaxSlices + 1] = {};
    uint32_t xs_edge_end[kMaxSlices] = {};
    // push engine (built on first use): out-edge destinations and weights in CSR order
    uint32_t* out_dst = nullptr;
    uint32_t* out_w = nullptr;
    bool out_built = false;
};

// Kernel view of a device graph.
struct GraphArgs {
    uint32_t n;
    uint32_t m;
    uint32_t rows;
    const uint32_t* __restrict__ in_src;
    const uint32_t* __restrict__ in_w;
    const uint64_t* __restrict__ rowmask;
    const uint32_t* __restrict__ rowseg;
    const uint32_t* __restrict__ nzdst;
#ifdef WEDGE_DEBUG_CHECKS
    const uint32_t* __restrict__ col_off;  // checks that a lane's (position, destination) is an in-edge
#endif
};

inline GraphArgs args_of(const DevGraph& g) {
    GraphArgs a;
    a.n = g.n;
    a.m = (uint32_t)g.m;
    a.rows = (uint32_t)g.rows;
    a.in_src = g.in_src;
    a.in_w = g.in_w;
    a.rowmask = g.rowmask;
    a.rowseg = g.rowseg;
    a.nzdst = g.nzdst;
#ifdef WEDGE_DEBUG_CHECKS
    a.col_off = g.col_off;
#endif
    return a;
}

// Kernel view of the source-sliced copy (positions over all slices, padded).
inline GraphArgs xs_args_of(const DevGraph& g) {
    GraphArgs a;
    a.n = g.n;
    a.m = (uint32_t)g.xs_positions;
    a.rows = (uint32_t)g.xs_rows;
    a.in_src = g.xs_src;
    a.in_w = g.xs_w;
    a.rowmask = g.xs_rowmask;
    a.rowseg = g.xs_rowseg;
    a.nzdst = g.xs_nzdst;
#ifdef WEDGE_DEBUG_CHECKS
    a.col_off = nullptr;  // positions are not canonical in-edge positions
#endif
    return a;
}

// 64-lane slots needed to cover K chunks of 2^lc positions.
#if defined(__HIPCC__)
__host__ __device__
#endif
inline uint64_t chunk_slots_count(uint64_t K, int lc) {
    return lc <= 6 ? (K + (64u >> lc) - 1) / (64u >> lc) : K << (lc - 6);
}

// Learned-gate sizes: 8 features -> 32 -> 32 -> 4 predicted log-times.
constexpr int kMlpIn = 8, kMlpHidden = 32, kMlpOut = 4;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpOut * kMlpHidden + kMlpOut;  // 1476
constexpr uint32_t kMlpMaxMembers = 8;  // ensemble size limit

// Decision state of the device-side gate, carried across iterations.
struct GateState {
    unsigned long long stamp;  // wall clock at the start of the current iteration
    uint32_t k;                // index of the iteration being decided
    uint32_t prev_mode;        // mode index of the previous iteration (0 full, 1..3 Wedge 16/32/64)
    uint32_t mode;             // decision: 1 Wedge Frontier, 0 full pull
    uint32_t lc;               // decision: log2 of edges per Wedge bit
    uint32_t learned;          // decisions taken by the model
    uint32_t fallback;         // decisions taken by the threshold rule
    uint32_t pad[2];
};

// Iteration counters written by the kernels and read back by the host.
struct Ctl {
    unsigned long long fnext;  // (listed count << 33) | out-degree sum of the next frontier
    unsigned long long marked; // (chunks appended to the chunk list) << 33
    unsigned long long ftotal; // next-frontier size, including vertices without out-edges
    GateState gate;
};
static_assert(sizeof(Ctl) == 64, "counter block layout");

constexpr int kDegBits = 33;
constexpr unsigned long long kDegMask = (1ull << kDegBits) - 1;

// Control block of the persistent traversal kernel (device memory). The
// barrier's words sit on cache lines of their own: the generation (polled by
// every waiting block), the top-level arrival counter, and one arrival counter
// per block group, so that arrivals of different groups do not serialise on
// one address. Words written by plain stores (the iteration count, the
// counter blocks) have lines of their own too. Iteration k reads its frontier
// counters from cnt[k & 1]; its commit writes cnt[(k + 1) & 1].
constexpr int kBarGroups = 16;
constexpr int kLineWords = 32;  // 128-byte lines of 4-byte words
struct alignas(128) CtlLine {
    Ctl c;
};
struct PersistState {
    unsigned bar_gen;        // grid barrier generation
    unsigned error;          // set when a barrier wait passed its deadline
    unsigned pad0[kLineWords - 2];
    unsigned bar_top[kLineWords];                // [0]: groups arrived
    unsigned bar_grp[kBarGroups][kLineWords];    // [g][0]: blocks of group g arrived
    unsigned iters;          // iterations run
    unsigned not_converged;  // stopped by max_iters with a non-empty frontier
    unsigned pad1[kLineWords - 2];
    CtlLine cnt[2];
};
static_assert(sizeof(CtlLine) == 128 && sizeof(PersistState) % 128 == 0, "persistent state layout");

struct PersistParams {
    GraphArgs g;
    uint32_t n;
    const uint32_t* row_off;
    const uint32_t* pos;
    uint32_t* level;            // single-level BFS values (internal order)
    uint64_t* visited;          // multi-source masks
    uint64_t* masks[2];
    uint32_t* lev;              // multi-source levels, lev[v*K + s]
    uint32_t K;
    uint64_t all;               // mask of the K sources
    uint64_t* fbits;
    uint64_t* fcur;
    uint32_t* flist[2];
    uint32_t* degpre[2];
    uint64_t* wbits;
    uint64_t wwords;
    uint32_t* chunks;
    int lc;
    PersistState* ps;
    wedge_iter_record* trace;
    uint32_t trace_cap;
    uint64_t thr;
    uint32_t gate;
    uint32_t max_iters;
    uint64_t timeout_ticks;
};

struct Workspace {
    uint32_t n = 0;
    uint64_t m = 0;
    uint64_t* fbits = nullptr;     // ceil(n/64) words: next-frontier bitmap (kept all-zero between uses)
    uint64_t* fcur = nullptr;      // ceil(n/64) words: current-frontier bitmap
    uint32_t* val = nullptr;       // n: values in internal order (relabelled graphs)
    uint32_t* flist[2] = {nullptr, nullptr};
    uint32_t* degpre[2] = {nullptr, nullptr};
    uint32_t* val_prev = nullptr;  // n
    uint64_t* wbits = nullptr;     // ceil(ceil(m/chunk)/64) words for the smallest chunk so far
    uint64_t wbits_words = 0;
    uint32_t* fsum = nullptr;      // summary flags of fbits (kept all-zero between uses)
    uint32_t* csum = nullptr;      // summary flags of fcur
    uint32_t* wsum = nullptr;      // summary flags of wbits (sized with it)
    uint32_t* chunks = nullptr;    // chunk list
    uint64_t chunks_cap = 0;
    Ctl* ctl = nullptr;            // device counters
    Ctl* ctl_host = nullptr;       // pinned mirror (host address)
    Ctl* ctl_host_dev = nullptr;   // its device address (written by launch_publish_ctl)
    // sequence number the publishing kernel writes after the counters (host
    // memory, in the same allocation): the host waits for it instead of the
    // stream
    volatile uint64_t* seq_host = nullptr;
    uint64_t* seq_dev = nullptr;
    uint64_t seq = 0;
    // PageRank
    float* pr_sum = nullptr;       // n
    float* pr_contrib = nullptr;   // n
    float* pr_rank = nullptr;      // n: ranks in internal order (relabelled graphs)
    float* pr_head = nullptr;      // tiles
    float* pr_tail = nullptr;      // tiles
    double* pr_part = nullptr;     // per-block dangling partials
    double* pr_d = nullptr;        // [2] dangling mass
    uint64_t pr_tiles = 0;
    uint32_t pr_parts = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // batched BFS
    uint64_t* visited = nullptr;   // n multi-source masks
    uint64_t* masks[2] = {nullptr, nullptr};
    uint32_t* lev = nullptr;       // n * lev_k multi-source levels
    uint32_t lev_k = 0;
    uint32_t* roots = nullptr;     // device copy of sources / roots
    uint32_t* roots_host = nullptr;// pinned staging
    uint32_t roots_cap = 0;
    PersistState* ps = nullptr;
    PersistState* ps_host = nullptr;
    wedge_iter_record* trace = nullptr;
    wedge_iter_record* trace_host = nullptr;
    uint32_t trace_cap = 0;
    uint64_t generation = 0;       // bumped whenever a buffer above moves
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    std::string graph_key;
};

}  // namespace wedge

// Learned-gate model: FP32 parameters, the training envelope of each feature,
// and their device copies (made on first use on a GPU).
struct wedge_model_s {
    uint32_t members = 1;        // ensemble size (1 .. kMlpMaxMembers)
    std::vector<float> params;   // members x kMlpParams, each W1 b1 W2 b2 W3 b3 (row-major out x in)
    std::vector<float> lo, hi;   // per-feature envelope
    float margin = 0.f;          // decision margin over the threshold rule (mean log-time units)
    float* dev_params = nullptr;
    float* dev_lo = nullptr;
    float* dev_hi = nullptr;
    int device = -1;
    bool dirty = true;           // host copy changed since the last upload
};

struct wedge_graph_s {
    uint32_t flags = 0;
    bool weighted = false;
    bool host_only = false;
    uint32_t dangling = 0;
    uint32_t max_w = 0;
    wedge::HostLayout host;        // kept only for WEDGE_HOST_ONLY graphs
    std::vector<uint32_t> perm_host;  // original -> internal id (empty: identity)
    std::vector<uint64_t> parts;      // batch graphs: first vertex of each part (+ total)
    wedge::DevGraph dev;
    wedge::Workspace ws;
    uint64_t device_bytes = 0;
    int device = 0;
    std::mutex busy;
};

namespace wedge {

// Records msg as the thread's last error and returns st.
wedge_status set_error(wedge_status st, const std::string& msg);

// One process-wide lock around the library's calls that are not stream
// ordered (hipMalloc, hipFree, synchronous memsets, pinned allocations, event
// creation, module symbol lookup) and around its stream captures: such a call
// made by one thread while another thread's stream is being captured can
// invalidate that capture, so the two never overlap. Recursive, because the
// setup paths nest.
std::recursive_mutex& setup_mutex();
struct SetupLock {
    std::lock_guard<std::recursive_mutex> guard{setup_mutex()};
};
// Uploads the model to the current device if needed.
wedge_status model_to_device(wedge_model_s* m);

// ------------------------------------------------------ kernel launchers
// (kernels.hip). Every launcher enqueues on `s` and returns the launch status.
hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s);
// Zero up to kClearMax device regions (16-byte aligned starts, sizes in
// 4-byte words) in one launch: one kernel instead of a runtime fill per
// buffer.
constexpr int kClearMax = 8;
struct ClearList {
    uint32_t* p[kClearMax] = {};
    uint64_t words[kClearMax] = {};
    int count = 0;
    void add(void* ptr, uint64_t bytes) {
        if (ptr && bytes) { p[count] = static_cast<uint32_t*>(ptr); words[count] = bytes / 4; ++count; }
    }
};
hipError_t launch_clear(const ClearList& l, hipStream_t s);
// Copy the counter block into host memory the device can write (host_dev:
// its device address; null: no copy), when `clear` zero the three
// accumulated counters for the next iteration, then (seq_dev non-null) store
// `seq` into host memory once the copy is visible to the host.
hipError_t launch_publish_ctl(Ctl* ctl, Ctl* host_dev, bool clear, uint64_t* seq_dev, uint64_t seq,
                              hipStream_t s);
hipError_t launch_iota_u32(uint32_t* p, uint32_t count, hipStream_t s);
// Summaries (fsum of the next-frontier bitmap, csum of the current one, wsum of
// the Wedge bitmap): one 32-bit flag per 4096 bits, set by every writer of a
// bit in that range and cleared by the compaction that lists it; nullable
// (null: the compaction scans every word and no flag is kept).
constexpr uint32_t kSumBits = 4096;
inline uint64_t sum_flags(uint64_t bits) { return (bits + kSumBits - 1) / kSumBits; }
hipError_t launch_seed_source(uint32_t src, const uint32_t* row_off, uint32_t* val_a,
                              uint32_t* val_b, uint32_t* flist, uint32_t* degpre, uint64_t* fcur,
                              uint32_t* csum, Ctl* ctl, hipStream_t s);
hipError_t launch_seed_all(uint32_t n, uint64_t m, const uint32_t* row_off, const uint32_t* inv,
                           uint32_t* label, uint32_t* val_prev, uint32_t* flist, uint32_t* degpre,
                           uint64_t* fcur, uint32_t* csum, Ctl* ctl, hipStream_t s);
hipError_t launch_unpermute_u32(uint32_t n, const uint32_t* perm, const uint32_t* val,
                                uint32_t* out, hipStream_t s);
hipError_t launch_unpermute_f32(uint32_t n, const uint32_t* perm, const float* val, float* out,
                                hipStream_t s);
hipError_t launch_set_f64(double* p, double v, hipStream_t s);
hipError_t launch_translate(const uint32_t* flist, const uint32_t* degpre, uint32_t fcount,
                            uint64_t active, const uint32_t* row_off, const uint32_t* pos,
                            int log_chunk, uint64_t* wbits, uint32_t* wsum, hipStream_t s);
hipError_t launch_compact_chunks(uint64_t* wbits, uint64_t words, uint32_t* list, Ctl* ctl,
                                 uint32_t* wsum, hipStream_t s);
// rows: 64-edge rows per wave step, 4, 8 or 16 for BFS, 8 for CC and SSSP
// (anything else returns hipErrorInvalidValue before any launch).
// inplace (CC and SSSP): gather sources' values from val instead of val_prev.
// Full pulls set no next-frontier bits: finalise such an iteration with
// launch_finalize(..., from_values = true, iter + 1) (CC and SSSP, also in
// place, with val_prev holding the values the iteration started from).
hipError_t launch_pull_full(int app, const DevGraph& g, uint32_t iter, uint32_t* val,
                            const uint32_t* val_prev, const uint64_t* fcur, uint64_t* fbits,
                            uint32_t* fsum, hipStream_t s, int rows = kPullRows, bool inplace = false);
hipError_t launch_pull_chunks(int app, const DevGraph& g, uint32_t iter, int log_chunk,
                              const uint32_t* list, const Ctl* ctl, uint64_t max_chunks,
                              uint32_t* val, const uint32_t* val_prev, const uint64_t* fcur,
                              uint64_t* fbits, uint32_t* fsum, hipStream_t s, int rows = kPullRows,
                              bool inplace = false);
// Lists the next-frontier bitmap (with out-degree prefix), commits val to
// val_prev for listed vertices (when val_prev is set), moves the bitmap into
// fcur (when set) and clears it. from_values (after a full pull, which sets
// no bits; needs val and fcur): the next frontier is every vertex with val <
// val_prev (CC, SSSP) or, without val_prev, with val == level (BFS) instead.
hipError_t launch_finalize(uint64_t* fbits, uint32_t n, const uint32_t* row_off, uint32_t* flist,
                           uint32_t* degpre, Ctl* ctl, uint32_t* val_prev, const uint32_t* val,
                           uint64_t* fcur, uint32_t* fsum, uint32_t* csum, hipStream_t s,
                           bool from_values = false, uint32_t level = 0);
// PageRank
// PageRank contributions of a graph with the sliced copy are kept in
// slice-major order: vertex v at slice_of(v) * cap + slice_local(v), cap the
// slice-local id capacity (whole 1024-vertex groups), so that the sliced pull
// indexes them by the slice-local id its in-edge word holds. cap = 0: vertex
// order.
inline uint64_t xs_contrib_cap(const DevGraph& g) {
    if (!g.xs_rows) return 0;
    const uint64_t groups = ((uint64_t)g.n + (1u << kXcdGroupShift) - 1) >> kXcdGroupShift;
    const uint64_t per = (groups + (1u << g.xs_lg) - 1) >> g.xs_lg;
    return per << kXcdGroupShift;
}
hipError_t launch_pr_init(uint32_t n, const uint32_t* row_off, float* rank, float* contrib,
                          float* sum, hipStream_t s, uint32_t lg = 0, uint64_t cap = 0);
hipError_t launch_pr_pull(const DevGraph& g, const float* contrib, float* sum, float* head,
                          float* tail, int cus, hipStream_t s);
// Completes S for destinations crossing tile boundaries, and reduces the
// previous epilogue's dangling partials into *d_next (when d_next is set).
hipError_t launch_pr_fixup(const DevGraph& g, const float* head, const float* tail, float* sum,
                           const double* partials, uint32_t parts, double* d_next, hipStream_t s);
hipError_t launch_pr_epilogue(uint32_t n, const uint32_t* row_off, float* sum,
                              double damping, const double* d_cur, float* rank, float* contrib,
                              double* partials, uint32_t parts, hipStream_t s, uint32_t lg = 0,
                              uint64_t cap = 0);
uint32_t pr_epilogue_blocks(uint32_t n);
// Batched BFS (batch.hip)
hipError_t launch_ms_pull_full(const DevGraph& g, uint64_t all, const uint64_t* visited,
                               const uint64_t* cur, uint64_t* nxt, uint64_t* fbits, uint32_t* fsum,
                               hipStream_t s, int rows = kPullRows);
hipError_t launch_ms_pull_chunks(const DevGraph& g, int lc, const uint32_t* list, const Ctl* ctl,
                                 uint64_t max_chunks, uint64_t all, const uint64_t* visited,
                                 const uint64_t* cur, uint64_t* nxt, uint64_t* fbits, uint32_t* fsum,
                                 hipStream_t s, int rows = kPullRows);
// Commit of a multi-source iteration (see ms_finalize_block); `retire` holds
// the masks of the frontier being replaced, `nxt` those just built.
hipError_t launch_ms_finalize(uint64_t* fbits, uint32_t n, const uint32_t* row_off,
                              uint32_t* flist, uint32_t* degpre, Ctl* ctl, uint64_t* fcur,
                              uint64_t* visited, uint64_t* retire, const uint64_t* nxt,
                              uint32_t* lev, uint32_t K, uint32_t level, uint32_t* fsum,
                              uint32_t* csum, hipStream_t s);
hipError_t launch_ms_seed(const uint32_t* srcs, uint32_t K, uint64_t* nxt, uint64_t* fbits,
                          uint32_t* fsum, hipStream_t s);
hipError_t launch_roots_seed(const uint32_t* roots, uint32_t count, uint32_t* level,
                             uint64_t* fbits, uint32_t* fsum, hipStream_t s);
hipError_t launch_ms_output(uint32_t n, uint32_t K, const uint32_t* perm, const uint32_t* lev,
                            uint32_t* out, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t s);
hipError_t launch_fill_u32_kernel(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s);
hipError_t persistent_max_blocks(bool ms, int* blocks_per_cu);
// Learned gate (mlp.hip)
hipError_t launch_mlp_forward(const float* P, uint32_t members, const float* X, float* Y,
                              uint32_t count, hipStream_t s);
hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, const float* Mk,
                           uint32_t count, float scale, float* G, float* loss, hipStream_t s);
hipError_t launch_adam(float* P, float* G, float* M1, float* M2, float lr, float b1, float b2,
                       float eps, uint32_t step, hipStream_t s);
// P null: the threshold rule decides (no model)
hipError_t launch_mlp_infer(const float* P, uint32_t members, const float* lo, const float* hi,
                            float margin, Ctl* ctl, double n, double m, uint64_t thr,
                            uint32_t fallback_lc, double ticks_per_us, uint32_t app, hipStream_t s);
hipError_t launch_gate_stamp(Ctl* ctl, hipStream_t s);
// Host form of the gate features (same formula as the device).
void mlp_features(float* x, double fcount, double active, double n, double m, double k,
                  double prev_us, double prev_mode, double app);
hipError_t launch_bfs_persistent(bool ms, const PersistParams& P, uint32_t blocks, hipStream_t s);

// Push engine (push.hip): the out-edge arrays from the edge index, and one
// push iteration over the listed frontier (val_prev: committed values, CC and
// SSSP; out_w: SSSP).
hipError_t launch_out_edges(const DevGraph& g, const uint32_t* pos, uint32_t* out_dst, uint32_t* out_w,
                            hipStream_t s);
hipError_t launch_push(int app, const uint32_t* flist, const uint32_t* degpre, uint32_t fcount,
                       uint64_t active, const uint32_t* row_off, const uint32_t* out_dst,
                       const uint32_t* out_w, uint32_t iter, uint32_t* val, const uint32_t* val_prev,
                       uint64_t* fbits, uint32_t* fsum, hipStream_t s);

// Debug builds (WEDGE_DEBUG_CHECKS): each kernel source keeps an error word
// that failed device checks OR their codes into; these read and clear them
// (0 in other builds).
hipError_t debug_take_kernels(unsigned* word);
hipError_t debug_take_batch(unsigned* word);
hipError_t debug_take_push(unsigned* word);
constexpr unsigned kDbgPullPos = 1u, kDbgPullDst = 2u, kDbgPullEdge = 4u, kDbgTranslate = 8u,
                   kDbgChunk = 16u;

// Allocation-free BFS (noalloc.hip): the fixed device scratch of each GPU,
// looked up once per device (dev must be the current device), and the lock
// that runs its users one at a time per device.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
constexpr int kNoAllocMaxDevices = 64;
hipError_t noalloc_scratch(int dev, void** ptr);
std::mutex& noalloc_run_lock(int dev);  // dev in [0, kNoAllocMaxDevices)

}  // namespace wedge
