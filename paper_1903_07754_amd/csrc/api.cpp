// C ABI of the Wedge-Frontier pull engine: argument checks, graph upload, the
// per-iteration control loop (Wedge Overview, Fig. 5) and PageRank.
#include <algorithm>
#include <atomic>
#include <map>
#include <tuple>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "wedge_internal.h"

namespace wedge {
hipError_t launch_set_f64(double* p, double v, hipStream_t s);
}

using namespace wedge;

namespace {

thread_local std::string g_err;

// roctx range over a scope: runs and iterations show up as named phases in a
// marker trace (rocprofv3 --marker-trace); without a tool attached the calls
// do nothing.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

wedge_status fail(wedge_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

}  // namespace

namespace wedge {
wedge_status set_error(wedge_status st, const std::string& msg) { return fail(st, msg); }
std::recursive_mutex& setup_mutex() {
    static std::recursive_mutex mu;
    return mu;
}
}  // namespace wedge

namespace {

wedge_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return WEDGE_ERR_HIP;
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

uint64_t device_cap() {
    const char* e = std::getenv("WEDGE_MAX_DEVICE_BYTES");
    return e ? std::strtoull(e, nullptr, 10) : 0;
}

// Device allocation accounted against the graph (and the optional cap).
wedge_status dev_alloc(wedge_graph_s* g, void** p, size_t bytes, const char* what) {
    SetupLock lock;
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    uint64_t cap = device_cap();
    if (cap && g->device_bytes + bytes > cap)
        return fail(WEDGE_ERR_OOM, std::string("device memory cap (WEDGE_MAX_DEVICE_BYTES) exceeded by ") + what);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? WEDGE_ERR_OOM : WEDGE_ERR_HIP,
                    std::string("hipMalloc failed for ") + what + ": " + hipGetErrorString(e));
    }
    g->device_bytes += bytes;
    return WEDGE_OK;
}

template <class T>
wedge_status upload(wedge_graph_s* g, T** dst, const std::vector<T>& src, hipStream_t s,
                    const char* what) {
    wedge_status st = dev_alloc(g, (void**)dst, src.size() * sizeof(T), what);
    if (st != WEDGE_OK) return st;
    if (!src.empty())
        HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s), what);
    return WEDGE_OK;
}

void free_all(wedge_graph_s* g) {
    SetupLock lock;
    DevGraph& d = g->dev;
    void* ptrs[] = {d.col_off, d.in_src, d.in_w, d.row_off, d.pos, d.rowmask, d.rowseg, d.nzdst, d.spans,
                    d.perm, d.inv, d.out_dst, d.out_w, d.xs_src, d.xs_w, d.xs_rowmask, d.xs_rowseg,
                    d.xs_nzdst, d.xs_pspan_v, d.xs_pspan_off, d.xs_pspan_tt};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    Workspace& w = g->ws;
    void* wp[] = {w.fbits, w.fcur, w.flist[0], w.flist[1], w.degpre[0], w.degpre[1], w.val_prev,
                  w.val, w.wbits, w.chunks, w.ctl, w.pr_sum, w.pr_contrib, w.pr_rank, w.pr_head,
                  w.pr_tail, w.pr_part, w.pr_d, w.fsum, w.csum, w.wsum};
    for (void* p : wp)
        if (p) (void)hipFree(p);
    if (w.ctl_host) (void)hipHostFree(w.ctl_host);
    void* bp[] = {w.visited, w.masks[0], w.masks[1], w.lev, w.roots, w.ps, w.trace};
    for (void* p : bp)
        if (p) (void)hipFree(p);
    void* hp[] = {w.roots_host, w.ps_host, w.trace_host};
    for (void* p : hp)
        if (p) (void)hipHostFree(p);
    if (w.graph_exec) (void)hipGraphExecDestroy(w.graph_exec);
    if (w.graph) (void)hipGraphDestroy(w.graph);
    if (w.capture_stream) (void)hipStreamDestroy(w.capture_stream);
    for (hipEvent_t e : w.ev)
        if (e) (void)hipEventDestroy(e);
    d = DevGraph{};
    w = Workspace{};
}

bool is_pow2(uint32_t x) { return x && !(x & (x - 1)); }
int log2u(uint32_t x) { int l = 0; while ((1u << l) < x) ++l; return l; }

template <class T>
wedge_status copy_input(const T* p, uint64_t count, bool on_device, std::vector<T>* tmp,
                        const T** out) {
    if (!p || !on_device) { *out = p; return WEDGE_OK; }
    tmp->resize(count ? count : 1);
    HIP_TRY(hipMemcpy(tmp->data(), p, count * sizeof(T), hipMemcpyDeviceToHost), "copying input graph");
    *out = tmp->data();
    return WEDGE_OK;
}

int device_cus(int dev);

// Whether a graph gets the source-sliced in-edge copy (WEDGE_SLICED_PULL).
bool sliced_pull_wanted(uint64_t m) {
    const char* e = std::getenv("WEDGE_SLICED_PULL");
    if (e && *e) return e[0] == '1';
    return m >= (1ull << 22);
}

wedge_status create(bool from_csr, uint32_t n, uint64_t m, const uint64_t* off, const uint32_t* ids,
                    const uint32_t* w, uint32_t flags, hipStream_t stream, wedge_graph_t* out) {
    if (!out) return fail(WEDGE_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (flags & ~(WEDGE_INPUT_DEVICE | WEDGE_SYMMETRIZE | WEDGE_HOST_ONLY | WEDGE_KEEP_IDS))
        return fail(WEDGE_ERR_INVALID_ARG, "unknown flag bits");
    if ((flags & WEDGE_HOST_ONLY) && (flags & WEDGE_INPUT_DEVICE))
        return fail(WEDGE_ERR_INVALID_ARG, "WEDGE_HOST_ONLY cannot take device input");
    if (n >= (1u << 31)) return fail(WEDGE_ERR_BAD_GRAPH, "n must be < 2^31");
    if (m >= (1ull << 32)) return fail(WEDGE_ERR_BAD_GRAPH, "m must be < 2^32");
    if (!off) return fail(WEDGE_ERR_INVALID_ARG, "offsets pointer is null");
    if (m && !ids) return fail(WEDGE_ERR_INVALID_ARG, "edge array pointer is null");
    const bool on_dev = flags & WEDGE_INPUT_DEVICE;
    std::vector<uint64_t> toff;
    std::vector<uint32_t> tids, tw;
    const uint64_t* hoff = nullptr;
    const uint32_t *hids = nullptr, *hw = nullptr;
    wedge_status st;
    if ((st = copy_input(off, (uint64_t)n + 1, on_dev, &toff, &hoff)) != WEDGE_OK) return st;
    if ((st = copy_input(ids, m, on_dev, &tids, &hids)) != WEDGE_OK) return st;
    if ((st = copy_input(w, m, on_dev, &tw, &hw)) != WEDGE_OK) return st;
    auto* g = new wedge_graph_s();
    g->flags = flags;
    g->host_only = flags & WEDGE_HOST_ONLY;
    HostLayout& L = g->host;
    const bool sym = flags & WEDGE_SYMMETRIZE;
    const bool relabel = !(flags & WEDGE_KEEP_IDS);
    st = from_csr ? build_layout_from_csr(n, m, hoff, hids, hw, sym, relabel, &L, &g_err)
                  : build_layout_from_csc(n, m, hoff, hids, hw, sym, relabel, &L, &g_err);
    if (st != WEDGE_OK) { delete g; return st; }
    if (sliced_pull_wanted(L.m)) build_xcd_slices(&L);
    g->weighted = !L.in_w.empty() || (w != nullptr);
    g->dangling = L.dangling;
    g->max_w = L.max_w;
    DevGraph& d = g->dev;
    d.n = L.n;
    d.m = L.m;
    d.rows = (L.m + 63) / 64;
    d.nonempty = (uint32_t)L.nzdst.size();
    d.nspans = L.spans.size() / 3;
    d.short_spans = L.short_spans;
    if (!L.xs_rowmask.empty() && L.xs_row_begin[1u << L.xs_lg]) {
        d.xs_lg = L.xs_lg;
        d.xs_rows = L.xs_row_begin[1u << L.xs_lg];
        d.xs_positions = d.xs_rows * 64;
        d.xs_segments = L.xs_nzdst.size();
        std::memcpy(d.xs_row_begin, L.xs_row_begin, sizeof d.xs_row_begin);
        std::memcpy(d.xs_edge_end, L.xs_edge_end, sizeof d.xs_edge_end);
        d.xs_packed = L.xs_packed;
        d.xs_pspans = L.xs_pspan_v.size();
        d.xs_pspan_short = L.xs_pspan_short;
        d.xs_pspan_pairs = L.xs_pspan_tt.size() / 2;
    }
    g->perm_host = L.perm;
    if (g->host_only) { *out = g; return WEDGE_OK; }
    {
        const hipError_t e = hipGetDevice(&g->device);
        if (e != hipSuccess) { delete g; return hip_fail(e, "hipGetDevice"); }
        d.cus = device_cus(g->device);
    }
    st = WEDGE_OK;
    SetupLock upload_lock;
    if (st == WEDGE_OK) st = upload(g, &d.col_off, L.col_off, stream, "col_off");
    // the in-edge arrays go up extended to whole rows plus kRowPad rows (zeros:
    // vertex 0, weight 0), so the full pulls read every lane of a wave's rows
    // without clamping
    auto to_whole_rows = [](std::vector<uint32_t> a) {
        a.resize(((a.size() + 63) / 64 + kRowPad) * 64, 0u);
        return a;
    };
    const std::vector<uint32_t> in_src_p = to_whole_rows(L.in_src);
    const std::vector<uint32_t> in_w_p = g->weighted ? to_whole_rows(L.in_w) : std::vector<uint32_t>();
    if (st == WEDGE_OK) st = upload(g, &d.in_src, in_src_p, stream, "in_src");
    if (st == WEDGE_OK && g->weighted) st = upload(g, &d.in_w, in_w_p, stream, "in_w");
    if (st == WEDGE_OK) st = upload(g, &d.row_off, L.row_off, stream, "row_off");
    if (st == WEDGE_OK) st = upload(g, &d.pos, L.pos, stream, "pos");
    // the row layouts go up with kRowPad rows of padding: the full pulls read
    // a few rows past the end instead of clamping (a mask of 1 and the last
    // segment index, which keep those rows' destination reads in bounds)
    // (the padded copies live until the stream is synchronised below)
    auto pad_masks = [](std::vector<uint64_t> mk) {
        mk.insert(mk.end(), kRowPad, 1ull);
        return mk;
    };
    auto pad_segs = [](std::vector<uint32_t> sg, size_t nz) {
        sg.insert(sg.end(), kRowPad, nz ? (uint32_t)(nz - 1) : 0u);
        return sg;
    };
    const std::vector<uint64_t> rowmask_p = pad_masks(L.rowmask);
    const std::vector<uint32_t> rowseg_p = pad_segs(L.rowseg, L.nzdst.size());
    const std::vector<uint64_t> xs_rowmask_p = d.xs_rows ? pad_masks(L.xs_rowmask) : std::vector<uint64_t>();
    const std::vector<uint32_t> xs_rowseg_p =
        d.xs_rows ? pad_segs(L.xs_rowseg, L.xs_nzdst.size()) : std::vector<uint32_t>();
    if (st == WEDGE_OK) st = upload(g, &d.rowmask, rowmask_p, stream, "rowmask");
    if (st == WEDGE_OK) st = upload(g, &d.rowseg, rowseg_p, stream, "rowseg");
    if (st == WEDGE_OK) st = upload(g, &d.nzdst, L.nzdst, stream, "nzdst");
    if (st == WEDGE_OK) st = upload(g, &d.spans, L.spans, stream, "spans");
    if (st == WEDGE_OK && !L.perm.empty()) st = upload(g, &d.perm, L.perm, stream, "perm");
    if (st == WEDGE_OK && !L.inv.empty()) st = upload(g, &d.inv, L.inv, stream, "inv");
    const std::vector<uint32_t> xs_src_p = d.xs_rows ? to_whole_rows(L.xs_src) : std::vector<uint32_t>();
    const std::vector<uint32_t> xs_w_p = d.xs_rows && !L.xs_w.empty() ? to_whole_rows(L.xs_w) : std::vector<uint32_t>();
    if (st == WEDGE_OK && d.xs_rows) st = upload(g, &d.xs_src, xs_src_p, stream, "sliced in-edges");
    if (st == WEDGE_OK && d.xs_rows && !L.xs_w.empty()) st = upload(g, &d.xs_w, xs_w_p, stream, "sliced weights");
    if (st == WEDGE_OK && d.xs_rows) st = upload(g, &d.xs_rowmask, xs_rowmask_p, stream, "sliced row masks");
    if (st == WEDGE_OK && d.xs_rows) st = upload(g, &d.xs_rowseg, xs_rowseg_p, stream, "sliced row segments");
    if (st == WEDGE_OK && d.xs_rows) st = upload(g, &d.xs_nzdst, L.xs_nzdst, stream, "sliced segment destinations");
    if (st == WEDGE_OK && d.xs_pspans) st = upload(g, &d.xs_pspan_v, L.xs_pspan_v, stream, "sliced PageRank spans");
    if (st == WEDGE_OK && d.xs_pspans) st = upload(g, &d.xs_pspan_off, L.xs_pspan_off, stream, "sliced PageRank span offsets");
    if (st == WEDGE_OK && d.xs_pspans) st = upload(g, &d.xs_pspan_tt, L.xs_pspan_tt, stream, "sliced PageRank span tiles");
    if (st == WEDGE_OK) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) st = hip_fail(e, "uploading graph");
    }
    if (st != WEDGE_OK) {
        (void)hipStreamSynchronize(stream);  // no upload may still read host data or write freed memory
        free_all(g);
        delete g;
        return st;
    }
    g->host = HostLayout{};  // device graph: drop the host copy
    *out = g;
    return WEDGE_OK;
}

// ----------------------------------------------------------- workspace

wedge_status ensure_workspace(wedge_graph_s* g, int log_chunk, bool need_frontier, bool need_chunks) {
    SetupLock lock;
    Workspace& w = g->ws;
    const DevGraph& d = g->dev;
    wedge_status st;
    // every buffer is allocated on its own when missing, so a run after a
    // failed (partial) allocation completes the workspace instead of using it.
    // Any buffer that is (re)allocated here moves, so the generation is bumped:
    // a captured persistent traversal holds the old addresses and must be
    // recorded again.
    auto need = [&](void** p, size_t bytes, const char* what) -> wedge_status {
        if (*p) return WEDGE_OK;
        w.generation++;
        return dev_alloc(g, p, bytes, what);
    };
    if ((st = need((void**)&w.ctl, sizeof(Ctl), "counters")) != WEDGE_OK) return st;
    if (!w.ctl_host) {
        // coherent: the device writes the counters straight into it
        // the counter block, then the publishing sequence number
        HIP_TRY(hipHostMalloc((void**)&w.ctl_host, 2 * sizeof(Ctl), hipHostMallocCoherent), "pinned counters");
        void* dp = nullptr;
        const hipError_t e = hipHostGetDevicePointer(&dp, w.ctl_host, 0);
        if (e != hipSuccess) {
            (void)hipHostFree(w.ctl_host);
            w.ctl_host = nullptr;
            return hip_fail(e, "mapping pinned counters");
        }
        w.ctl_host_dev = static_cast<Ctl*>(dp);
        w.seq_host = reinterpret_cast<volatile uint64_t*>(w.ctl_host + 1);
        w.seq_dev = reinterpret_cast<uint64_t*>(w.ctl_host_dev + 1);
        *w.seq_host = 0;
        w.seq = 0;
    }
    for (auto& e : w.ev)
        if (!e) HIP_TRY(hipEventCreate(&e), "event");
    if (need_frontier) {
        w.n = d.n;
        w.m = d.m;
        const uint64_t fw = ((uint64_t)d.n + 63) / 64;
        if (!w.fbits) {
            w.generation++;
            if ((st = dev_alloc(g, (void**)&w.fbits, fw * 8, "frontier bitmap")) != WEDGE_OK) return st;
            HIP_TRY(hipMemset(w.fbits, 0, fw ? fw * 8 : 8), "clearing frontier bitmap");
        }
        if ((st = need((void**)&w.fcur, fw * 8, "current frontier bitmap")) != WEDGE_OK) return st;
        if (!w.fsum) {
            w.generation++;
            if ((st = dev_alloc(g, (void**)&w.fsum, sum_flags(d.n) * 4, "frontier summary")) != WEDGE_OK) return st;
            HIP_TRY(hipMemset(w.fsum, 0, sum_flags(d.n) * 4), "clearing frontier summary");
        }
        if ((st = need((void**)&w.csum, sum_flags(d.n) * 4, "current frontier summary")) != WEDGE_OK) return st;
        if (d.inv && (st = need((void**)&w.val, (size_t)d.n * 4, "values")) != WEDGE_OK) return st;
        for (int i = 0; i < 2; ++i) {
            if ((st = need((void**)&w.flist[i], (size_t)d.n * 4, "frontier list")) != WEDGE_OK) return st;
            if ((st = need((void**)&w.degpre[i], (size_t)d.n * 4, "degree prefix")) != WEDGE_OK) return st;
        }
        if ((st = need((void**)&w.val_prev, (size_t)d.n * 4, "committed values")) != WEDGE_OK) return st;
    }
    if (need_chunks) {
        const uint64_t chunks = (d.m + (1ull << log_chunk) - 1) >> log_chunk;
        const uint64_t words = (chunks + 63) / 64;
        if (words > w.wbits_words || !w.wbits || !w.wsum) {
            w.generation++;
            if (w.wbits) { (void)hipFree(w.wbits); g->device_bytes -= w.wbits_words * 8; w.wbits = nullptr; }
            if (w.wsum) { (void)hipFree(w.wsum); g->device_bytes -= sum_flags(w.wbits_words * 64) * 4; w.wsum = nullptr; }
            w.wbits_words = 0;
            const uint64_t alloc_words = words ? words : 1;
            if ((st = dev_alloc(g, (void**)&w.wbits, alloc_words * 8, "Wedge Frontier bitmap")) != WEDGE_OK) return st;
            w.wbits_words = alloc_words;
            HIP_TRY(hipMemset(w.wbits, 0, w.wbits_words * 8), "clearing Wedge bitmap");
            const uint64_t flags = sum_flags(w.wbits_words * 64);
            if ((st = dev_alloc(g, (void**)&w.wsum, flags * 4, "Wedge Frontier summary")) != WEDGE_OK) return st;
            HIP_TRY(hipMemset(w.wsum, 0, flags * 4), "clearing Wedge summary");
        }
        if (chunks > w.chunks_cap || !w.chunks) {
            w.generation++;
            if (w.chunks) { (void)hipFree(w.chunks); g->device_bytes -= w.chunks_cap * 4; w.chunks = nullptr; }
            if ((st = dev_alloc(g, (void**)&w.chunks, chunks * 4, "chunk list")) != WEDGE_OK) return st;
            w.chunks_cap = chunks ? chunks : 2;
        }
    }
    return WEDGE_OK;
}

struct RunGuard {
    std::mutex& m;
    bool ok;
    explicit RunGuard(std::mutex& mu) : m(mu), ok(mu.try_lock()) {}
    ~RunGuard() { if (ok) m.unlock(); }
};

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

const wedge_opts kDefaultOpts = {WEDGE_GATE_THRESHOLD, 0, 0, 0, 0, 0, nullptr, nullptr, 0, 0};

wedge_status check_run(wedge_graph_t g, const void* out, const wedge_opts* o) {
    if (!g) return fail(WEDGE_ERR_INVALID_ARG, "graph is null");
    if (g->host_only) return fail(WEDGE_ERR_UNSUPPORTED, "graph was created with WEDGE_HOST_ONLY");
    if (!out && g->dev.n) return fail(WEDGE_ERR_INVALID_ARG, "output pointer is null");
    if (o->gate > WEDGE_GATE_HYBRID) return fail(WEDGE_ERR_INVALID_ARG, "unknown gate");
    if (o->chunk_edges && (!is_pow2(o->chunk_edges) || o->chunk_edges > 4096))
        return fail(WEDGE_ERR_INVALID_ARG, "chunk_edges must be a power of two in [1, 4096]");
    if (o->trace_cap && !o->trace) return fail(WEDGE_ERR_INVALID_ARG, "trace_cap set but trace is null");
    if (o->flags & ~(WEDGE_RUN_TIME_PULL | WEDGE_RUN_TIME_ITERS | WEDGE_RUN_PERSISTENT | WEDGE_RUN_INPLACE))
        return fail(WEDGE_ERR_INVALID_ARG, "unknown run flag bits");
    if (o->rows_per_wave && o->rows_per_wave != 4 && o->rows_per_wave != 8 && o->rows_per_wave != 16)
        return fail(WEDGE_ERR_INVALID_ARG, "rows_per_wave must be 0, 4, 8 or 16");
    return WEDGE_OK;
}

// Pull shapes other than the default exist for the host-driven BFS kinds only.
wedge_status check_rows(const wedge_opts& o, bool shaped) {
    if (o.rows_per_wave && o.rows_per_wave != (uint32_t)kPullRows && !shaped)
        return fail(WEDGE_ERR_UNSUPPORTED,
                    "rows_per_wave other than 8 applies to host-driven BFS, multi-source and batch runs");
    return WEDGE_OK;
}

wedge_status run_bfs_roots(wedge_graph_t g, const uint32_t* roots, uint32_t count, uint32_t* out,
                           const wedge_opts* opts_in, hipStream_t s, wedge_stats* stats);

bool push_gate(uint32_t gate) { return gate == WEDGE_GATE_ALWAYS_PUSH || gate == WEDGE_GATE_HYBRID; }

// Gates that may build the Wedge Frontier (and so need its bitmap and list).
bool wedge_gate_used(uint32_t gate) { return gate != WEDGE_GATE_ALWAYS_FULL && !push_gate(gate); }

// The push engine's out-edge arrays, built once per graph on the device from
// the edge index and the row layout.
wedge_status ensure_push(wedge_graph_s* g, hipStream_t s) {
    SetupLock lock;
    DevGraph& d = g->dev;
    if (d.out_built) return WEDGE_OK;
    wedge_status st;
    if (!d.out_dst && (st = dev_alloc(g, (void**)&d.out_dst, (size_t)d.m * 4, "push out-edges")) != WEDGE_OK)
        return st;
    if (d.in_w && !d.out_w && (st = dev_alloc(g, (void**)&d.out_w, (size_t)d.m * 4, "push weights")) != WEDGE_OK)
        return st;
    HIP_TRY(launch_out_edges(d, d.pos, d.out_dst, d.out_w, s), "building push out-edges");
    HIP_TRY(hipStreamSynchronize(s), "building push out-edges");
    d.out_built = true;
    return WEDGE_OK;
}

// ------------------------------------------------------------ the loop
//
// The control loop of one traversal (Wedge Overview, Fig. 5): with the
// frontier's size, listed count and A read back from the device, choose the
// mode, build the Wedge Frontier when chosen, pull, finalise, repeat until the
// frontier is empty. The app supplies the pull and finalise launches.
// Engine of one iteration (the mode recorded in wedge_iter_record).
constexpr int kModeFull = 0, kModeWedge = 1, kModePush = 2;
// Default threshold of the hybrid baseline: 5% of the edges.
constexpr uint32_t kHybridThetaPpm = 50000;

// Default fullness threshold per application (Evaluation, Frontier Fullness
// Threshold: theta is tuned per machine by timing iterations with and without
// the Wedge Frontier). BFS 1% and CC 20% are the paper's values, which a
// sweep on this GPU confirms; for SSSP the same sweep gives 5% (faster than
// 20% on every graph swept: the sliced full pull beats marked-chunk pulls
// that cover most of the edges).
uint32_t default_theta_ppm(int app) { return app == kBfs ? 10000u : app == kCc ? 200000u : 50000u; }

struct LoopCfg {
    int lc = 5;
    uint64_t thr = 0;
    uint32_t gate = WEDGE_GATE_THRESHOLD;
    uint32_t max_iters = 0;
    bool time_pull = false, time_iter = false;
    uint64_t nchunks = 0, wwords = 0;
    // learned gate: decisions come from the device (model may be null: threshold rule)
    bool learned = false;
    const float* P = nullptr;
    uint32_t members = 1;
    const float* lo = nullptr;
    const float* hi = nullptr;
    float margin = 0.f;
    double ticks_per_us = 100.0;
    uint64_t m = 0;
    uint32_t app = kBfs;       // application (a gate feature)
    int rows = kPullRows;      // pull shape: 64-edge rows per wave step
    // values the push engine updates and reads (push and hybrid gates)
    uint32_t* val = nullptr;
    const uint32_t* val_prev = nullptr;
    // the smallest chunk exponent this run may use (bitmap and list sizes)
    int min_lc() const { return learned ? std::min(lc, 4) : lc; }
    uint64_t chunks_of(int l) const { return (m + (1ull << l) - 1) >> l; }
};

// Enqueue the copy of the counter block to the host (complete once the stream
// is synchronised) and, when `clear`, the zeroing of its accumulated counters.
// Workspaces without device-writable host memory (the allocation-free entry
// point) copy with the runtime instead.
hipError_t read_counters(Workspace& w, bool clear, hipStream_t s) {
    if (w.ctl_host_dev) return launch_publish_ctl(w.ctl, w.ctl_host_dev, clear, w.seq_dev, ++w.seq, s);
    hipError_t e = hipMemcpyAsync(w.ctl_host, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && clear) e = launch_publish_ctl(w.ctl, nullptr, true, nullptr, 0, s);
    return e;
}

// Wait until the counters enqueued by read_counters are in host memory. With
// the publishing kernel the host polls the sequence number it stores last (a
// stream synchronisation wakes the host some tens of microseconds later);
// every few thousand polls the stream is queried, so a failed launch ends the
// wait with its error. Without it, the stream is synchronised.
hipError_t wait_counters(Workspace& w, hipStream_t s) {
    if (!w.seq_host) return hipStreamSynchronize(s);
    for (uint64_t polls = 1;; ++polls) {
        if (*w.seq_host == w.seq) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return hipSuccess;
        }
        if ((polls & 4095u) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return e;
            // the stream has drained: the sequence number must be there now
            if (*w.seq_host == w.seq) {
                std::atomic_thread_fence(std::memory_order_acquire);
                return hipSuccess;
            }
            return hipErrorUnknown;
        }
    }
}

template <class Pull, class Fin>
wedge_status iterate(wedge_graph_t g, Workspace& w, const wedge_opts& o, const LoopCfg& c,
                     hipStream_t s, wedge_stats& local, double t0, wedge_stats* stats, Pull pull,
                     Fin fin) {
    const DevGraph& d = g->dev;
    if (c.learned)
        HIP_TRY(launch_mlp_infer(c.P, c.members, c.lo, c.hi, c.margin, w.ctl, (double)d.n, (double)d.m, c.thr, (uint32_t)c.lc,
                                 c.ticks_per_us, c.app, s), "gate inference");
    // the counters come back through host memory the device writes; the
    // publishing kernel also clears them for the next iteration (the learned
    // gate's stamp kernel clears them instead)
    HIP_TRY(read_counters(w, !c.learned, s), "reading counters");
    HIP_TRY(wait_counters(w, s), "initialising run");
    uint64_t fcount = w.ctl_host->ftotal;               // |F_k|
    uint64_t flisted = w.ctl_host->fnext >> kDegBits;   // of which have out-edges
    uint64_t active = w.ctl_host->fnext & kDegMask;     // A_k
    int cur = 0;
    uint32_t k = 0;
    for (; fcount > 0; ++k) {
        if (k >= c.max_iters) {
            local.iterations = k;
            if (stats) { local.ms = now_ms() - t0; *stats = local; }
            return fail(WEDGE_ERR_NOT_CONVERGED, "max_iters reached with a non-empty frontier");
        }
        int mode;  // kModeFull, kModeWedge or kModePush
        int lc = c.lc;
        if (c.learned) {
            mode = w.ctl_host->gate.mode != 0 ? kModeWedge : kModeFull;
            lc = (int)w.ctl_host->gate.lc;
        } else {
            switch (c.gate) {
                case WEDGE_GATE_ALWAYS_WEDGE: mode = kModeWedge; break;
                case WEDGE_GATE_ALWAYS_FULL: mode = kModeFull; break;
                case WEDGE_GATE_ALWAYS_PUSH: mode = kModePush; break;
                // the hybrid engine: push below the threshold, else the full pull
                case WEDGE_GATE_HYBRID: mode = active < c.thr ? kModePush : kModeFull; break;
                default: mode = active < c.thr ? kModeWedge : kModeFull; break;  // strict <
            }
        }
        const bool wedge_mode = mode == kModeWedge;
        Range iter_range(mode == kModeWedge ? "wedge iteration"
                         : mode == kModePush ? "push iteration" : "full-pull iteration");
        if (c.learned) HIP_TRY(launch_gate_stamp(w.ctl, s), "clearing counters");
        if (c.time_iter) HIP_TRY(hipEventRecord(w.ev[2], s), "event");
        uint64_t maxk = 0;
        if (wedge_mode) {
            const uint64_t nch = c.chunks_of(lc);
            HIP_TRY(launch_translate(w.flist[cur], w.degpre[cur], (uint32_t)flisted, active, d.row_off,
                                     d.pos, lc, w.wbits, w.wsum, s), "frontier translation");
            HIP_TRY(launch_compact_chunks(w.wbits, (nch + 63) / 64, w.chunks, w.ctl, w.wsum, s), "chunk compaction");
            maxk = active < nch ? active : nch;
        }
        if (c.time_pull) HIP_TRY(hipEventRecord(w.ev[0], s), "event");
        if (mode == kModePush)
            HIP_TRY(launch_push(c.app, w.flist[cur], w.degpre[cur], (uint32_t)flisted, active, d.row_off,
                                d.out_dst, d.out_w, k, c.val, c.val_prev, w.fbits, w.fsum, s), "push");
        else
            HIP_TRY(pull(k, wedge_mode, maxk, cur, lc), wedge_mode ? "chunk pull" : "full pull");
        if (c.time_pull) HIP_TRY(hipEventRecord(w.ev[1], s), "event");
        HIP_TRY(fin(k, cur), "frontier finalisation");
        if (c.time_iter) HIP_TRY(hipEventRecord(w.ev[3], s), "event");
        if (c.learned)
            HIP_TRY(launch_mlp_infer(c.P, c.members, c.lo, c.hi, c.margin, w.ctl, (double)d.n, (double)d.m, c.thr,
                                     (uint32_t)c.lc, c.ticks_per_us, c.app, s), "gate inference");
        HIP_TRY(read_counters(w, !c.learned, s), "reading counters");
        HIP_TRY(wait_counters(w, s), "iteration");
        float pms = 0.f, ims = 0.f;
        // the events precede the publishing kernel: done on the device, and
        // waited for here so that the runtime has taken their completion
        if (c.time_pull) HIP_TRY(hipEventSynchronize(w.ev[1]), "event");
        if (c.time_iter) HIP_TRY(hipEventSynchronize(w.ev[3]), "event");
        if (c.time_pull) HIP_TRY(hipEventElapsedTime(&pms, w.ev[0], w.ev[1]), "event time");
        if (c.time_iter) HIP_TRY(hipEventElapsedTime(&ims, w.ev[2], w.ev[3]), "event time");
        local.pull_ms += pms;
        local.pull_launches++;
        if (mode == kModeFull) {
            local.full_pull_ms += pms;
            local.full_pull_launches++;
        }
        const uint64_t marked = wedge_mode ? (w.ctl_host->marked >> kDegBits) : 0;
        if (o.trace && k < o.trace_cap) {
            wedge_iter_record& r = o.trace[k];
            r.iter = k;
            r.mode = (uint32_t)mode;
            r.chunk_edges = wedge_mode ? (1u << lc) : 0u;
            r.reserved = 0;
            r.frontier = fcount;
            r.active_edges = active;
            r.marked_chunks = marked;
            r.ms = ims;
            r.reserved2 = 0.f;
        }
        if (mode == kModeWedge) { local.wedge_iters++; local.edges_scanned += marked << lc; }
        else if (mode == kModePush) { local.push_iters++; local.edges_scanned += active; }
        else { local.full_iters++; local.edges_scanned += d.m; }
        fcount = w.ctl_host->ftotal;
        flisted = w.ctl_host->fnext >> kDegBits;
        active = w.ctl_host->fnext & kDegMask;
        cur ^= 1;
    }
    local.iterations = k;
    return WEDGE_OK;
}

LoopCfg loop_cfg(const wedge_opts& o, const DevGraph& d, App app, uint32_t theta_default,
                 uint32_t chunk_default) {
    LoopCfg c;
    c.app = (uint32_t)app;
    const uint32_t theta = o.threshold_ppm ? o.threshold_ppm
                                           : (o.gate == WEDGE_GATE_HYBRID ? kHybridThetaPpm : theta_default);
    const uint32_t chunk = o.chunk_edges ? o.chunk_edges : chunk_default;
    c.lc = log2u(chunk);
    c.thr = ((uint64_t)theta * d.m) / 1000000ull;
    c.gate = o.gate;
    c.max_iters = o.max_iters ? o.max_iters : d.n + 1;
    c.rows = o.rows_per_wave ? (int)o.rows_per_wave : kPullRows;
    c.time_pull = o.flags & WEDGE_RUN_TIME_PULL;
    c.time_iter = o.flags & WEDGE_RUN_TIME_ITERS;
    c.nchunks = (d.m + chunk - 1) >> c.lc;
    c.wwords = (c.nchunks + 63) / 64;
    c.m = d.m;
    if (o.gate == WEDGE_GATE_LEARNED) {
        c.learned = true;
        const wedge_model_s* md = static_cast<const wedge_model_s*>(o.model);
        if (md && md->dev_params) {
            c.P = md->dev_params;
            c.members = md->members;
            c.lo = md->dev_lo;
            c.hi = md->dev_hi;
            c.margin = md->margin;
        }
    }
    return c;
}

double wall_ticks_per_us(int dev) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;
    return (double)khz / 1000.0;
}

// Learned gate: upload the model (if any) and fill the device pointers.
wedge_status prepare_gate(wedge_graph_t g, const wedge_opts& o, LoopCfg* c) {
    if (!c->learned) return WEDGE_OK;
    c->ticks_per_us = wall_ticks_per_us(g->device);
    if (o.model) {
        wedge_model_s* md = const_cast<wedge_model_s*>(static_cast<const wedge_model_s*>(o.model));
        wedge_status st = model_to_device(md);
        if (st != WEDGE_OK) return st;
        c->P = md->dev_params;
        c->members = md->members;
        c->lo = md->dev_lo;
        c->hi = md->dev_hi;
        c->margin = md->margin;
    }
    return WEDGE_OK;
}

// Clears both frontier bitmaps (and the Wedge bitmap when it may be used)
// and the counter block, in one launch.
wedge_status clear_bitmaps(wedge_graph_t g, const LoopCfg& c, hipStream_t s) {
    const Workspace& w = g->ws;
    const uint64_t fwords = ((uint64_t)g->dev.n + 63) / 64;
    ClearList l;
    l.add(w.fbits, fwords * 8);
    l.add(w.fcur, fwords * 8);
    l.add(w.fsum, sum_flags(g->dev.n) * 4);
    l.add(w.csum, sum_flags(g->dev.n) * 4);
    l.add(w.ctl, sizeof(Ctl));
    if (wedge_gate_used(c.gate)) {
        const uint64_t words = (c.chunks_of(c.min_lc()) + 63) / 64;
        l.add(w.wbits, words * 8);
        l.add(w.wsum, sum_flags(words * 64) * 4);
    }
    HIP_TRY(launch_clear(l, s), "clearing bitmaps and counters");
    return WEDGE_OK;
}

// BFS, CC and SSSP from one source (or all vertices for CC).
wedge_status run_frontier_app(int app, wedge_graph_t g, uint32_t src, uint32_t* val,
                              const wedge_opts* opts_in, hipStream_t s, wedge_stats* stats) {
    Range run_range(app == kBfs ? "wedge_bfs" : app == kCc ? "wedge_cc" : "wedge_sssp");
    const wedge_opts& o = opts_in ? *opts_in : kDefaultOpts;
    wedge_status st = check_run(g, val, &o);
    if (st != WEDGE_OK) return st;
    const DevGraph& d = g->dev;
    if (app != kCc && src >= d.n) return fail(WEDGE_ERR_INVALID_ARG, "source vertex out of range");
    if (app == kSssp) {
        if (!g->weighted) return fail(WEDGE_ERR_NO_WEIGHTS, "SSSP needs a graph created with weights");
        if (d.n && (uint64_t)(d.n - 1) * g->max_w >= 0xFFFFFFFFull)
            return fail(WEDGE_ERR_INVALID_ARG, "(n-1) * max weight must be < 2^32 - 1");
    }
    if (app == kCc && !(g->flags & WEDGE_SYMMETRIZE))
        return fail(WEDGE_ERR_UNSUPPORTED, "CC runs on the undirected view: create the graph with WEDGE_SYMMETRIZE");
    const bool inplace = o.flags & WEDGE_RUN_INPLACE;
    if (inplace && (app == kBfs || push_gate(o.gate)))
        return fail(WEDGE_ERR_UNSUPPORTED, "the in-place pull applies to CC and SSSP with pull gates");
    if (app == kBfs && (o.flags & WEDGE_RUN_PERSISTENT))
        return run_bfs_roots(g, &src, 1, val, opts_in, s, stats);
    if ((o.flags & WEDGE_RUN_PERSISTENT)) return fail(WEDGE_ERR_UNSUPPORTED, "persistent runs are BFS kinds only");
    if ((st = check_rows(o, app == kBfs)) != WEDGE_OK) return st;
    RunGuard guard(g->busy);
    if (!guard.ok) return fail(WEDGE_ERR_BUSY, "graph is in use by another run");
    wedge_stats local{};
    const double t0 = now_ms();
    if (d.n == 0) { if (stats) *stats = local; return WEDGE_OK; }
    LoopCfg c = loop_cfg(o, d, (App)app, default_theta_ppm(app), app == kBfs ? 32u : 16u);
    if ((st = prepare_gate(g, o, &c)) != WEDGE_OK) return st;
    if ((st = ensure_workspace(g, c.min_lc(), true, wedge_gate_used(c.gate))) != WEDGE_OK) return st;
    if (push_gate(c.gate) && (st = ensure_push(g, s)) != WEDGE_OK) return st;
    Workspace& w = g->ws;
    if ((st = clear_bitmaps(g, c, s)) != WEDGE_OK) return st;
    // values are computed in internal vertex order; a relabelled graph works in
    // a workspace array and is mapped to the caller's order at the end
    uint32_t* const out = val;
    if (d.inv) val = w.val;
    const uint32_t isrc = (app != kCc && !g->perm_host.empty()) ? g->perm_host[src] : src;
    uint32_t* vprev = app == kBfs ? nullptr : w.val_prev;
    c.val = val;
    c.val_prev = vprev;
    if (app == kCc) {
        HIP_TRY(launch_seed_all(d.n, d.m, d.row_off, d.inv, val, w.val_prev, w.flist[0], w.degpre[0],
                                w.fcur, w.csum, w.ctl, s), "seeding CC");
    } else {
        HIP_TRY(launch_fill_u32(val, d.n, kInf, s), "initialising values");
        if (vprev) HIP_TRY(launch_fill_u32(vprev, d.n, kInf, s), "initialising values");
        HIP_TRY(launch_seed_source(isrc, d.row_off, val, vprev, w.flist[0], w.degpre[0], w.fcur,
                                   w.csum, w.ctl, s), "seeding source");
    }
    // a full pull sets no bits: its finalisation takes the next frontier from
    // the values (val < val_prev, or val == k + 1 for BFS; set by the pull,
    // read by the finalisation of the same iteration)
    bool bits_from_values = false;
    st = iterate(
        g, w, o, c, s, local, t0, stats,
        [&](uint32_t k, bool wedge_mode, uint64_t maxk, int, int lc) {
            bits_from_values = !wedge_mode;
            return wedge_mode ? launch_pull_chunks(app, d, k, lc, w.chunks, w.ctl, maxk, val, vprev,
                                                   w.fcur, w.fbits, w.fsum, s, c.rows, inplace)
                              : launch_pull_full(app, d, k, val, vprev, w.fcur, w.fbits, w.fsum, s, c.rows, inplace);
        },
        [&](uint32_t k, int cur) {
            const bool fv = bits_from_values;
            bits_from_values = false;  // a push iteration runs no pull
            // the in-place pull gathers no committed values, but the committed
            // copy is kept: a full pull's next frontier is compared against it
            return launch_finalize(w.fbits, d.n, d.row_off, w.flist[cur ^ 1], w.degpre[cur ^ 1], w.ctl,
                                   vprev, val, w.fcur, w.fsum, w.csum, s, fv, k + 1);
        });
    if (st != WEDGE_OK) return st;
    if (d.inv) {
        HIP_TRY(launch_unpermute_u32(d.n, d.perm, val, out, s), "writing results");
        HIP_TRY(hipStreamSynchronize(s), "writing results");
    }
    local.ms = now_ms() - t0;
    if (stats) *stats = local;
    return WEDGE_OK;
}

// BFS with its whole workspace carved out of the library's fixed device
// scratch (noalloc.hip) instead of the graph's allocated workspace. The loop
// and the kernels are those of run_frontier_app; what differs is that no
// call here allocates or frees memory: buffers are cleared by fill kernels,
// the counters are read back into a host variable, and the options that need
// an allocation (the learned gate's device model, timing events, the
// persistent launch's buffers) are refused. One frontier list and prefix
// serve both iterations' roles: the translation reads them before the pull,
// and the finalisation rewrites them after it, in stream order.
struct NoAllocPlan {
    uint64_t fwords, wwords, nchunks, fflags, wflags;
    size_t off_fbits, off_fcur, off_flist, off_degpre, off_val, off_wbits, off_chunks, off_ctl;
    size_t off_fsum, off_csum, off_wsum, total;
};

NoAllocPlan noalloc_plan(const DevGraph& d, const LoopCfg& c) {
    NoAllocPlan p{};
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    p.fwords = ((uint64_t)d.n + 63) / 64;
    p.nchunks = c.chunks_of(c.lc);
    p.wwords = (p.nchunks + 63) / 64;
    size_t at = 0;
    p.off_ctl = at;    at += up(sizeof(Ctl));
    p.off_fbits = at;  at += up(p.fwords * 8);
    p.off_fcur = at;   at += up(p.fwords * 8);
    p.off_flist = at;  at += up((size_t)d.n * 4);
    p.off_degpre = at; at += up((size_t)d.n * 4);
    p.off_val = at;    at += d.inv ? up((size_t)d.n * 4) : 0;
    p.off_wbits = at;  at += up((p.wwords ? p.wwords : 1) * 8);
    p.off_chunks = at; at += up((p.nchunks ? p.nchunks : 1) * 4);
    p.fflags = sum_flags(d.n);
    p.wflags = sum_flags((p.wwords ? p.wwords : 1) * 64);
    p.off_fsum = at;   at += up(p.fflags * 4);
    p.off_csum = at;   at += up(p.fflags * 4);
    p.off_wsum = at;   at += up(p.wflags * 4);
    p.total = at;
    return p;
}

wedge_status run_bfs_noalloc(wedge_graph_t g, uint32_t src, uint32_t* out, const wedge_opts* opts_in,
                             hipStream_t s, wedge_stats* stats) {
    const wedge_opts& o = opts_in ? *opts_in : kDefaultOpts;
    wedge_status st = check_run(g, out, &o);
    if (st != WEDGE_OK) return st;
    const DevGraph& d = g->dev;
    if (src >= d.n) return fail(WEDGE_ERR_INVALID_ARG, "source vertex out of range");
    if (o.gate == WEDGE_GATE_LEARNED)
        return fail(WEDGE_ERR_UNSUPPORTED, "the learned gate needs device model buffers: use wedge_bfs");
    if (push_gate(o.gate))
        return fail(WEDGE_ERR_UNSUPPORTED, "the push engine builds out-edge arrays on first use: use wedge_bfs");
    if (o.flags)
        return fail(WEDGE_ERR_UNSUPPORTED,
                    "timing and persistent runs need events or graph buffers: use wedge_bfs");
    if ((st = check_rows(o, true)) != WEDGE_OK) return st;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != g->device) return fail(WEDGE_ERR_INVALID_ARG, "the graph's device must be the current device");
    if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(WEDGE_ERR_UNSUPPORTED, "device index beyond the scratch table");
    const LoopCfg c = loop_cfg(o, d, kBfs, 10000u, 32u);
    const NoAllocPlan p = noalloc_plan(d, c);
    if (p.total > kNoAllocScratchBytes)
        return fail(WEDGE_ERR_INVALID_ARG,
                    "graph needs " + std::to_string(p.total) + " bytes of BFS workspace; the fixed scratch holds " +
                        std::to_string(kNoAllocScratchBytes) + " (use wedge_bfs)");
    RunGuard guard(g->busy);
    if (!guard.ok) return fail(WEDGE_ERR_BUSY, "graph is in use by another run");
    std::lock_guard<std::mutex> one_at_a_time(noalloc_run_lock(dev));
    void* base = nullptr;
    HIP_TRY(noalloc_scratch(dev, &base), "looking up the device scratch");
    unsigned char* b = static_cast<unsigned char*>(base);
    Workspace w{};
    Ctl host_ctl{};
    w.n = d.n;
    w.m = d.m;
    w.ctl = reinterpret_cast<Ctl*>(b + p.off_ctl);
    w.ctl_host = &host_ctl;
    w.fbits = reinterpret_cast<uint64_t*>(b + p.off_fbits);
    w.fcur = reinterpret_cast<uint64_t*>(b + p.off_fcur);
    w.flist[0] = w.flist[1] = reinterpret_cast<uint32_t*>(b + p.off_flist);
    w.degpre[0] = w.degpre[1] = reinterpret_cast<uint32_t*>(b + p.off_degpre);
    w.val = d.inv ? reinterpret_cast<uint32_t*>(b + p.off_val) : nullptr;
    w.wbits = reinterpret_cast<uint64_t*>(b + p.off_wbits);
    w.wbits_words = p.wwords;
    w.chunks = reinterpret_cast<uint32_t*>(b + p.off_chunks);
    w.chunks_cap = p.nchunks;
    w.fsum = reinterpret_cast<uint32_t*>(b + p.off_fsum);
    w.csum = reinterpret_cast<uint32_t*>(b + p.off_csum);
    w.wsum = reinterpret_cast<uint32_t*>(b + p.off_wsum);
    wedge_stats local{};
    const double t0 = now_ms();
    // the scratch keeps the previous call's contents: clear what must start at zero
    HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(w.ctl), sizeof(Ctl) / 8, 0, s), "clearing counters");
    HIP_TRY(launch_fill_u64(w.fbits, p.fwords, 0, s), "clearing frontier bitmap");
    HIP_TRY(launch_fill_u64(w.fcur, p.fwords, 0, s), "clearing frontier bitmap");
    HIP_TRY(launch_fill_u32_kernel(w.fsum, p.fflags, 0, s), "clearing frontier summary");
    HIP_TRY(launch_fill_u32_kernel(w.csum, p.fflags, 0, s), "clearing frontier summary");
    if (c.gate != WEDGE_GATE_ALWAYS_FULL) {
        HIP_TRY(launch_fill_u64(w.wbits, p.wwords, 0, s), "clearing Wedge bitmap");
        HIP_TRY(launch_fill_u32_kernel(w.wsum, p.wflags, 0, s), "clearing Wedge summary");
    }
    uint32_t* val = d.inv ? w.val : out;
    const uint32_t isrc = g->perm_host.empty() ? src : g->perm_host[src];
    HIP_TRY(launch_fill_u32(val, d.n, kInf, s), "initialising values");
    HIP_TRY(launch_seed_source(isrc, d.row_off, val, nullptr, w.flist[0], w.degpre[0], w.fcur, w.csum, w.ctl, s),
            "seeding source");
    bool bits_from_values = false;  // a full pull sets no bits (see run_frontier_app)
    st = iterate(
        g, w, o, c, s, local, t0, stats,
        [&](uint32_t k, bool wedge_mode, uint64_t maxk, int, int lc) {
            bits_from_values = !wedge_mode;
            return wedge_mode ? launch_pull_chunks(kBfs, d, k, lc, w.chunks, w.ctl, maxk, val, nullptr,
                                                   w.fcur, w.fbits, w.fsum, s, c.rows)
                              : launch_pull_full(kBfs, d, k, val, nullptr, w.fcur, w.fbits, w.fsum, s, c.rows);
        },
        [&](uint32_t k, int cur) {
            const bool fv = bits_from_values;
            bits_from_values = false;
            return launch_finalize(w.fbits, d.n, d.row_off, w.flist[cur ^ 1], w.degpre[cur ^ 1], w.ctl,
                                   nullptr, val, w.fcur, w.fsum, w.csum, s, fv, k + 1);
        });
    if (st != WEDGE_OK) {
        (void)hipStreamSynchronize(s);  // the next user of the scratch must not meet this run's kernels
        return st;
    }
    if (d.inv) HIP_TRY(launch_unpermute_u32(d.n, d.perm, val, out, s), "writing results");
    HIP_TRY(hipStreamSynchronize(s), "writing results");
    local.ms = now_ms() - t0;
    if (stats) *stats = local;
    return WEDGE_OK;
}

// ---------------------------------------------------------------- batching

wedge_status ensure_batch(wedge_graph_t g, uint32_t nroots, uint32_t K) {
    SetupLock lock;
    Workspace& w = g->ws;
    const DevGraph& d = g->dev;
    wedge_status st;
    // as in ensure_workspace, each buffer is (re)allocated on its own, and a
    // capacity is only raised once its buffers exist
    auto need = [&](void** p, size_t bytes, const char* what) -> wedge_status {
        return *p ? WEDGE_OK : dev_alloc(g, p, bytes, what);
    };
    if (nroots > w.roots_cap) {
        if (w.roots) { (void)hipFree(w.roots); g->device_bytes -= (uint64_t)w.roots_cap * 4; w.roots = nullptr; }
        if (w.roots_host) { (void)hipHostFree(w.roots_host); w.roots_host = nullptr; }
        w.roots_cap = 0;
        if ((st = dev_alloc(g, (void**)&w.roots, (size_t)nroots * 4, "sources")) != WEDGE_OK) return st;
        HIP_TRY(hipHostMalloc((void**)&w.roots_host, (size_t)nroots * 4, hipHostMallocDefault), "pinned sources");
        w.roots_cap = nroots;
        w.generation++;
    }
    if (K && !(w.visited && w.masks[0] && w.masks[1])) {
        if ((st = need((void**)&w.visited, (size_t)d.n * 8, "visited masks")) != WEDGE_OK) return st;
        for (int i = 0; i < 2; ++i)
            if ((st = need((void**)&w.masks[i], (size_t)d.n * 8, "frontier masks")) != WEDGE_OK) return st;
        w.generation++;
    }
    if (K > w.lev_k) {
        if (w.lev) { (void)hipFree(w.lev); g->device_bytes -= (uint64_t)d.n * w.lev_k * 4; w.lev = nullptr; }
        w.lev_k = 0;
        if ((st = dev_alloc(g, (void**)&w.lev, (size_t)d.n * K * 4, "multi-source levels")) != WEDGE_OK) return st;
        w.lev_k = K;
        w.generation++;
    }
    if (!(w.ps && w.ps_host && w.trace && w.trace_host)) {
        if ((st = need((void**)&w.ps, sizeof(PersistState), "persistent state")) != WEDGE_OK) return st;
        if (!w.ps_host)
            HIP_TRY(hipHostMalloc((void**)&w.ps_host, sizeof(PersistState), hipHostMallocDefault), "pinned state");
        w.trace_cap = 4096;
        if ((st = need((void**)&w.trace, (size_t)w.trace_cap * sizeof(wedge_iter_record), "trace")) != WEDGE_OK)
            return st;
        if (!w.trace_host)
            HIP_TRY(hipHostMalloc((void**)&w.trace_host, (size_t)w.trace_cap * sizeof(wedge_iter_record),
                                  hipHostMallocDefault), "pinned trace");
        w.generation++;
    }
    return WEDGE_OK;
}

// Copy the (caller-id) sources into the device buffer in internal ids.
wedge_status upload_roots(wedge_graph_t g, const uint32_t* roots, uint32_t count, hipStream_t s) {
    Workspace& w = g->ws;
    for (uint32_t i = 0; i < count; ++i)
        w.roots_host[i] = g->perm_host.empty() ? roots[i] : g->perm_host[roots[i]];
    if (count) HIP_TRY(hipMemcpyAsync(w.roots, w.roots_host, (size_t)count * 4, hipMemcpyHostToDevice, s), "uploading sources");
    return WEDGE_OK;
}

int device_cus(int dev) {
    static std::atomic<int> cache[64];
    if (dev >= 0 && dev < 64) {
        const int c = cache[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
        return 0;
    if (dev >= 0 && dev < 64) cache[dev].store(c, std::memory_order_relaxed);
    return c;
}

uint64_t barrier_timeout_ticks(int dev) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;
    double ms = 10000.0;  // a traversal step never waits this long on a healthy device
    if (const char* e = std::getenv("WEDGE_BARRIER_TIMEOUT_MS")) ms = std::strtod(e, nullptr);
    return (uint64_t)(ms * (double)khz);
}

// The persistent form of a BFS-kind traversal, recorded in a hipGraph (on a
// library stream: the legacy default stream cannot be captured) and replayed
// on the caller's stream.
wedge_status run_persistent(wedge_graph_t g, bool ms, uint32_t count, uint32_t* out,
                            const wedge_opts& o, const LoopCfg& c, hipStream_t s,
                            wedge_stats& local) {
    Workspace& w = g->ws;
    const DevGraph& d = g->dev;
    int bpc_max = 0;
    HIP_TRY(persistent_max_blocks(ms, &bpc_max), "occupancy query");
    if (bpc_max <= 0) return fail(WEDGE_ERR_UNSUPPORTED, "persistent kernel cannot be resident");
    const int cus = device_cus(g->device);
    if (cus <= 0) return fail(WEDGE_ERR_HIP, "cannot read the compute unit count");
    const uint32_t bpc = o.blocks_per_cu ? std::min<uint32_t>(o.blocks_per_cu, (uint32_t)bpc_max)
                                         : (uint32_t)bpc_max;
    const uint32_t blocks = bpc * (uint32_t)cus;
    uint32_t* level = d.inv ? w.val : out;
    const uint64_t timeout = barrier_timeout_ticks(g->device);
    char keybuf[256];
    std::snprintf(keybuf, sizeof keybuf, "%d|%u|%p|%u|%u|%d|%llu|%u|%llu|%llu", ms ? 1 : 0, count,
                  (void*)out, blocks, c.gate, c.lc, (unsigned long long)c.thr, c.max_iters,
                  (unsigned long long)w.generation, (unsigned long long)timeout);
    const std::string key(keybuf);
    if (key != w.graph_key || !w.graph_exec) {
        SetupLock capture_lock;
        if (w.graph_exec) { (void)hipGraphExecDestroy(w.graph_exec); w.graph_exec = nullptr; }
        if (w.graph) { (void)hipGraphDestroy(w.graph); w.graph = nullptr; }
        w.graph_key.clear();
        if (!w.capture_stream) HIP_TRY(hipStreamCreateWithFlags(&w.capture_stream, hipStreamNonBlocking), "capture stream");
        hipStream_t cs = w.capture_stream;
        PersistParams P{};
        P.g = args_of(d);
        P.n = d.n;
        P.row_off = d.row_off;
        P.pos = d.pos;
        P.level = level;
        P.visited = w.visited;
        P.masks[0] = w.masks[0];
        P.masks[1] = w.masks[1];
        P.lev = w.lev;
        P.K = ms ? count : 0;
        P.all = ms ? (count == 64 ? ~0ull : ((1ull << count) - 1ull)) : 0ull;
        P.fbits = w.fbits;
        P.fcur = w.fcur;
        P.flist[0] = w.flist[0];
        P.flist[1] = w.flist[1];
        P.degpre[0] = w.degpre[0];
        P.degpre[1] = w.degpre[1];
        P.wbits = w.wbits;
        P.wwords = c.wwords;
        P.chunks = w.chunks;
        P.lc = c.lc;
        P.ps = w.ps;
        P.trace = w.trace;
        P.trace_cap = w.trace_cap;
        P.thr = c.thr;
        P.gate = c.gate;
        P.max_iters = c.max_iters;
        P.timeout_ticks = timeout;
        const uint64_t fwords = ((uint64_t)d.n + 63) / 64;
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "graph capture");
        hipError_t e = hipSuccess;
        // every buffer is reset by kernels (no memset nodes in the graph)
        if (e == hipSuccess) e = launch_fill_u64(w.fbits, fwords, 0, cs);
        if (e == hipSuccess) e = launch_fill_u64(w.fcur, fwords, 0, cs);
        if (e == hipSuccess && c.gate != WEDGE_GATE_ALWAYS_FULL) e = launch_fill_u64(w.wbits, c.wwords, 0, cs);
        if (e == hipSuccess) e = launch_fill_u64(reinterpret_cast<uint64_t*>(w.ps), sizeof(PersistState) / 8, 0, cs);
        if (ms) {
            if (e == hipSuccess) e = launch_fill_u64(w.visited, d.n, 0, cs);
            if (e == hipSuccess) e = launch_fill_u64(w.masks[0], d.n, 0, cs);
            if (e == hipSuccess) e = launch_fill_u64(w.masks[1], d.n, 0, cs);
            if (e == hipSuccess) e = launch_fill_u32_kernel(w.lev, (uint64_t)d.n * count, kInf, cs);
            if (e == hipSuccess) e = launch_ms_seed(w.roots, count, w.masks[0], w.fbits, nullptr, cs);
        } else {
            if (e == hipSuccess) e = launch_fill_u32_kernel(level, d.n, kInf, cs);
            if (e == hipSuccess) e = launch_roots_seed(w.roots, count, level, w.fbits, nullptr, cs);
        }
        if (e == hipSuccess) e = launch_bfs_persistent(ms, P, blocks, cs);
        if (e == hipSuccess) {
            if (ms) e = launch_ms_output(d.n, count, d.perm, w.lev, out, cs);
            else if (d.inv) e = launch_unpermute_u32(d.n, d.perm, level, out, cs);
        }
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return hip_fail(e, "recording the persistent traversal"); }
        if (e2 != hipSuccess) return hip_fail(e2, "graph capture");
        w.graph = graph;
        HIP_TRY(hipGraphInstantiate(&w.graph_exec, w.graph, nullptr, nullptr, 0), "graph instantiation");
        w.graph_key = key;
    }
    {
        // The kernel's grid barriers need every block resident. Two persistent
        // grids on one device could each hold part of the CUs and wait for
        // blocks the other keeps out, so this process runs them one at a time
        // per device.
        static std::mutex device_mu[64];
        std::unique_lock<std::mutex> one_at_a_time;
        if (g->device >= 0 && g->device < 64) one_at_a_time = std::unique_lock<std::mutex>(device_mu[g->device]);
        HIP_TRY(hipGraphLaunch(w.graph_exec, s), "graph launch");
        HIP_TRY(hipMemcpyAsync(w.ps_host, w.ps, sizeof(PersistState), hipMemcpyDeviceToHost, s), "reading state");
        HIP_TRY(hipStreamSynchronize(s), "persistent traversal");
    }
    if (w.ps_host->error)
        return fail(WEDGE_ERR_HIP, "persistent traversal: a grid barrier passed its deadline "
                                   "(blocks not co-resident or WEDGE_BARRIER_TIMEOUT_MS too small)");
    const uint32_t iters = w.ps_host->iters;
    const uint32_t nrec = std::min(iters, w.trace_cap);
    if (nrec) {
        HIP_TRY(hipMemcpy(w.trace_host, w.trace, (size_t)nrec * sizeof(wedge_iter_record), hipMemcpyDeviceToHost), "reading trace");
    }
    for (uint32_t k = 0; k < nrec; ++k) {
        const wedge_iter_record& r = w.trace_host[k];
        if (r.mode) { local.wedge_iters++; local.edges_scanned += r.marked_chunks << c.lc; }
        else { local.full_iters++; local.edges_scanned += d.m; }
        if (o.trace && k < o.trace_cap) o.trace[k] = r;
    }
    local.iterations = iters;
    local.pull_launches = 1;
    if (w.ps_host->not_converged) return fail(WEDGE_ERR_NOT_CONVERGED, "max_iters reached with a non-empty frontier");
    return WEDGE_OK;
}

// BFS from every root at once (one traversal; with disjoint parts, the level
// of each vertex is the one from its own part's root).
wedge_status run_bfs_roots(wedge_graph_t g, const uint32_t* roots, uint32_t count, uint32_t* out,
                           const wedge_opts* opts_in, hipStream_t s, wedge_stats* stats) {
    Range run_range("wedge_bfs roots");
    const wedge_opts& o = opts_in ? *opts_in : kDefaultOpts;
    wedge_status st = check_run(g, out, &o);
    if (st != WEDGE_OK) return st;
    const DevGraph& d = g->dev;
    if (count && !roots) return fail(WEDGE_ERR_INVALID_ARG, "sources pointer is null");
    if (o.flags & WEDGE_RUN_INPLACE) return fail(WEDGE_ERR_UNSUPPORTED, "the in-place pull applies to CC and SSSP");
    for (uint32_t i = 0; i < count; ++i)
        if (roots[i] >= d.n) return fail(WEDGE_ERR_INVALID_ARG, "source vertex out of range");
    if ((st = check_rows(o, !(o.flags & WEDGE_RUN_PERSISTENT))) != WEDGE_OK) return st;
    RunGuard guard(g->busy);
    if (!guard.ok) return fail(WEDGE_ERR_BUSY, "graph is in use by another run");
    wedge_stats local{};
    const double t0 = now_ms();
    if (d.n == 0) { if (stats) *stats = local; return WEDGE_OK; }
    LoopCfg c = loop_cfg(o, d, kBfs, 10000u, 32u);
    if ((st = prepare_gate(g, o, &c)) != WEDGE_OK) return st;
    if ((o.flags & WEDGE_RUN_PERSISTENT) && c.learned)
        return fail(WEDGE_ERR_UNSUPPORTED, "the learned gate runs with the host-driven loop");
    if ((o.flags & WEDGE_RUN_PERSISTENT) && push_gate(c.gate))
        return fail(WEDGE_ERR_UNSUPPORTED, "the push engine runs with the host-driven loop");
    if ((st = ensure_workspace(g, c.min_lc(), true, true)) != WEDGE_OK) return st;
    if ((st = ensure_batch(g, count ? count : 1, 0)) != WEDGE_OK) return st;
    if (push_gate(c.gate) && (st = ensure_push(g, s)) != WEDGE_OK) return st;
    Workspace& w = g->ws;
    if ((st = upload_roots(g, roots, count, s)) != WEDGE_OK) return st;
    if (o.flags & WEDGE_RUN_PERSISTENT) {
        st = run_persistent(g, false, count, out, o, c, s, local);
    } else {
        if ((st = clear_bitmaps(g, c, s)) != WEDGE_OK) return st;
        uint32_t* val = d.inv ? w.val : out;
        c.val = val;
        HIP_TRY(launch_fill_u32(val, d.n, kInf, s), "initialising values");
        HIP_TRY(launch_roots_seed(w.roots, count, val, w.fbits, w.fsum, s), "seeding roots");
        HIP_TRY(launch_finalize(w.fbits, d.n, d.row_off, w.flist[0], w.degpre[0], w.ctl, nullptr, nullptr,
                                w.fcur, w.fsum, w.csum, s), "listing roots");
        bool bits_from_values = false;  // a full pull sets no bits (see run_frontier_app)
        st = iterate(
            g, w, o, c, s, local, t0, stats,
            [&](uint32_t k, bool wedge_mode, uint64_t maxk, int, int lc) {
                bits_from_values = !wedge_mode;
                return wedge_mode ? launch_pull_chunks(kBfs, d, k, lc, w.chunks, w.ctl, maxk, val,
                                                       nullptr, w.fcur, w.fbits, w.fsum, s, c.rows)
                                  : launch_pull_full(kBfs, d, k, val, nullptr, w.fcur, w.fbits, w.fsum, s, c.rows);
            },
            [&](uint32_t k, int cur) {
                const bool fv = bits_from_values;
                bits_from_values = false;
                return launch_finalize(w.fbits, d.n, d.row_off, w.flist[cur ^ 1], w.degpre[cur ^ 1],
                                       w.ctl, nullptr, val, w.fcur, w.fsum, w.csum, s, fv, k + 1);
            });
        if (st == WEDGE_OK && d.inv) {
            HIP_TRY(launch_unpermute_u32(d.n, d.perm, val, out, s), "writing results");
            HIP_TRY(hipStreamSynchronize(s), "writing results");
        }
    }
    local.ms = now_ms() - t0;
    if (stats) *stats = local;
    return st;
}

// Multi-source BFS with 64-bit masks.
wedge_status run_multisource(wedge_graph_t g, const uint32_t* srcs, uint32_t count, uint32_t* out,
                             const wedge_opts* opts_in, hipStream_t s, wedge_stats* stats) {
    Range run_range("wedge_bfs_multisource");
    const wedge_opts& o = opts_in ? *opts_in : kDefaultOpts;
    wedge_status st = check_run(g, out, &o);
    if (st != WEDGE_OK) return st;
    const DevGraph& d = g->dev;
    if (count < 1 || count > 64) return fail(WEDGE_ERR_INVALID_ARG, "count must be in [1, 64]");
    if (o.flags & WEDGE_RUN_INPLACE) return fail(WEDGE_ERR_UNSUPPORTED, "the in-place pull applies to CC and SSSP");
    if (!srcs) return fail(WEDGE_ERR_INVALID_ARG, "sources pointer is null");
    for (uint32_t i = 0; i < count; ++i)
        if (srcs[i] >= d.n) return fail(WEDGE_ERR_INVALID_ARG, "source vertex out of range");
    if ((st = check_rows(o, !(o.flags & WEDGE_RUN_PERSISTENT))) != WEDGE_OK) return st;
    if (push_gate(o.gate))
        return fail(WEDGE_ERR_UNSUPPORTED, "multi-source BFS has no push engine (use the threshold gate)");
    RunGuard guard(g->busy);
    if (!guard.ok) return fail(WEDGE_ERR_BUSY, "graph is in use by another run");
    wedge_stats local{};
    const double t0 = now_ms();
    if (d.n == 0) { if (stats) *stats = local; return WEDGE_OK; }
    LoopCfg c = loop_cfg(o, d, kBfs, 10000u, 32u);
    if ((st = prepare_gate(g, o, &c)) != WEDGE_OK) return st;
    if ((o.flags & WEDGE_RUN_PERSISTENT) && c.learned)
        return fail(WEDGE_ERR_UNSUPPORTED, "the learned gate runs with the host-driven loop");
    if ((st = ensure_workspace(g, c.min_lc(), true, true)) != WEDGE_OK) return st;
    if ((st = ensure_batch(g, count, count)) != WEDGE_OK) return st;
    Workspace& w = g->ws;
    if ((st = upload_roots(g, srcs, count, s)) != WEDGE_OK) return st;
    const uint64_t all = count == 64 ? ~0ull : ((1ull << count) - 1ull);
    if (o.flags & WEDGE_RUN_PERSISTENT) {
        st = run_persistent(g, true, count, out, o, c, s, local);
    } else {
        if ((st = clear_bitmaps(g, c, s)) != WEDGE_OK) return st;
        ClearList ml;
        ml.add(w.visited, (size_t)d.n * 8);
        ml.add(w.masks[0], (size_t)d.n * 8);
        ml.add(w.masks[1], (size_t)d.n * 8);
        HIP_TRY(launch_clear(ml, s), "clearing masks");
        HIP_TRY(launch_fill_u32_kernel(w.lev, (uint64_t)d.n * count, kInf, s), "initialising levels");
        HIP_TRY(launch_ms_seed(w.roots, count, w.masks[0], w.fbits, w.fsum, s), "seeding sources");
        HIP_TRY(launch_ms_finalize(w.fbits, d.n, d.row_off, w.flist[0], w.degpre[0], w.ctl, w.fcur,
                                   w.visited, w.masks[1], w.masks[0], w.lev, count, 0, w.fsum, w.csum, s), "listing sources");
        st = iterate(
            g, w, o, c, s, local, t0, stats,
            [&](uint32_t k, bool wedge_mode, uint64_t maxk, int, int lc) {
                const uint64_t* mc = w.masks[k & 1];
                uint64_t* mn = w.masks[(k & 1) ^ 1];
                return wedge_mode ? launch_ms_pull_chunks(d, lc, w.chunks, w.ctl, maxk, all, w.visited,
                                                          mc, mn, w.fbits, w.fsum, s, c.rows)
                                  : launch_ms_pull_full(d, all, w.visited, mc, mn, w.fbits, w.fsum, s, c.rows);
            },
            [&](uint32_t k, int cur) {
                return launch_ms_finalize(w.fbits, d.n, d.row_off, w.flist[cur ^ 1], w.degpre[cur ^ 1],
                                          w.ctl, w.fcur, w.visited, w.masks[k & 1],
                                          w.masks[(k & 1) ^ 1], w.lev, count, k + 1, w.fsum, w.csum, s);
            });
        if (st == WEDGE_OK) {
            HIP_TRY(launch_ms_output(d.n, count, d.perm, w.lev, out, s), "writing results");
            HIP_TRY(hipStreamSynchronize(s), "writing results");
        }
    }
    local.ms = now_ms() - t0;
    if (stats) *stats = local;
    return st;
}

// Debug builds: a run whose kernels failed a device check reports it (release
// builds read nothing).
wedge_status debug_verdict(wedge_status st) {
#ifdef WEDGE_DEBUG_CHECKS
    unsigned a = 0, b = 0, c = 0;
    if (debug_take_kernels(&a) != hipSuccess || debug_take_batch(&b) != hipSuccess ||
        debug_take_push(&c) != hipSuccess)
        return fail(WEDGE_ERR_HIP, "reading the device check words");
    if (a | b | c) {
        char msg[128];
        std::snprintf(msg, sizeof msg, "device check failed: codes 0x%x 0x%x 0x%x", a, b, c);
        return fail(WEDGE_ERR_HIP, msg);
    }
#endif
    return st;
}

}  // namespace

extern "C" {

wedge_status wedge_graph_create_csr(uint32_t n, uint64_t m, const uint64_t* row_off,
                                    const uint32_t* col, const uint32_t* w, uint32_t flags,
                                    hipStream_t stream, wedge_graph_t* out) {
    try {
        return create(true, n, m, row_off, col, w, flags, stream, out);
    } catch (const std::bad_alloc&) {
        return fail(WEDGE_ERR_OOM, "host allocation failed while building the layout");
    }
}

wedge_status wedge_graph_create_csc(uint32_t n, uint64_t m, const uint64_t* col_off,
                                    const uint32_t* src, const uint32_t* w, uint32_t flags,
                                    hipStream_t stream, wedge_graph_t* out) {
    try {
        return create(false, n, m, col_off, src, w, flags, stream, out);
    } catch (const std::bad_alloc&) {
        return fail(WEDGE_ERR_OOM, "host allocation failed while building the layout");
    }
}

wedge_status wedge_graph_destroy(wedge_graph_t g) {
    if (!g) return WEDGE_OK;
    if (!g->host_only) free_all(g);
    delete g;
    return WEDGE_OK;
}

wedge_status wedge_graph_get_info(wedge_graph_t g, wedge_graph_info* info) {
    if (!g || !info) return fail(WEDGE_ERR_INVALID_ARG, "null argument");
    info->n = g->dev.n;
    info->m = g->dev.m;
    info->nonempty = g->dev.nonempty;
    info->rows = g->dev.rows;
    info->flags = g->flags;
    info->weighted = g->weighted ? 1u : 0u;
    info->dangling = g->dangling;
    info->pr_tile_edges = 64u * kPrTileRows;
    info->pr_spans = g->dev.nspans;
    info->device_bytes = g->device_bytes;
    info->pr_short_spans = g->dev.short_spans;
    info->relabeled = g->perm_host.empty() ? 0u : 1u;
    info->xs_rows = g->dev.xs_rows;
    info->xs_slices = g->dev.xs_rows ? (1u << g->dev.xs_lg) : 0u;
    info->xs_segments = g->host_only ? g->host.xs_nzdst.size() : g->dev.xs_segments;
    info->xs_pr_spans = g->dev.xs_pspans;
    info->xs_pr_short_spans = g->dev.xs_pspan_short;
    info->xs_pr_span_pairs = g->dev.xs_pspan_pairs;
    info->xs_packed = g->dev.xs_packed ? 1u : 0u;
    return WEDGE_OK;
}

wedge_status wedge_graph_layout(wedge_graph_t g, wedge_layout_array which, void* dst,
                                uint64_t bytes) {
    if (!g || !dst) return fail(WEDGE_ERR_INVALID_ARG, "null argument");
    const DevGraph& d = g->dev;
    const HostLayout& L = g->host;
    const void* hsrc = nullptr;
    const void* dsrc = nullptr;
    uint64_t size = 0;
    switch (which) {
        case WEDGE_LAYOUT_COL_OFF: size = ((uint64_t)d.n + 1) * 4; hsrc = L.col_off.data(); dsrc = d.col_off; break;
        case WEDGE_LAYOUT_IN_SRC: size = d.m * 4; hsrc = L.in_src.data(); dsrc = d.in_src; break;
        case WEDGE_LAYOUT_IN_W:
            if (!g->weighted) return fail(WEDGE_ERR_NO_WEIGHTS, "graph has no weights");
            size = d.m * 4; hsrc = L.in_w.data(); dsrc = d.in_w; break;
        case WEDGE_LAYOUT_ROW_OFF: size = ((uint64_t)d.n + 1) * 4; hsrc = L.row_off.data(); dsrc = d.row_off; break;
        case WEDGE_LAYOUT_POS: size = d.m * 4; hsrc = L.pos.data(); dsrc = d.pos; break;
        case WEDGE_LAYOUT_ROWMASK: size = d.rows * 8; hsrc = L.rowmask.data(); dsrc = d.rowmask; break;
        case WEDGE_LAYOUT_ROWSEG: size = d.rows * 4; hsrc = L.rowseg.data(); dsrc = d.rowseg; break;
        case WEDGE_LAYOUT_NZDST: size = (uint64_t)d.nonempty * 4; hsrc = L.nzdst.data(); dsrc = d.nzdst; break;
        case WEDGE_LAYOUT_PR_SPANS: size = d.nspans * 12; hsrc = L.spans.data(); dsrc = d.spans; break;
        case WEDGE_LAYOUT_XS_SRC:
        case WEDGE_LAYOUT_XS_W:
        case WEDGE_LAYOUT_XS_ROWMASK:
        case WEDGE_LAYOUT_XS_ROWSEG:
        case WEDGE_LAYOUT_XS_NZDST:
        case WEDGE_LAYOUT_XS_PR_SPAN_V:
        case WEDGE_LAYOUT_XS_PR_SPAN_OFF:
        case WEDGE_LAYOUT_XS_PR_SPAN_TILES:
        case WEDGE_LAYOUT_XS_BOUNDS: {
            const uint64_t xr = d.xs_rows;
            const uint64_t xseg = g->host_only ? L.xs_nzdst.size() : d.xs_segments;
            if (!xr) return fail(WEDGE_ERR_UNSUPPORTED, "graph has no source-sliced in-edge copy");
            if (which == WEDGE_LAYOUT_XS_BOUNDS) {
                const int S = 1 << d.xs_lg;
                uint32_t b[2 * kMaxSlices + 1];
                for (int j = 0; j <= S; ++j) b[j] = d.xs_row_begin[j];
                for (int j = 0; j < S; ++j) b[S + 1 + j] = d.xs_edge_end[j];
                const uint64_t size = (uint64_t)(2 * S + 1) * 4;
                if (bytes != size) return fail(WEDGE_ERR_INVALID_ARG, "bytes does not match the array size");
                std::memcpy(dst, b, size);
                return WEDGE_OK;
            }
            if (which == WEDGE_LAYOUT_XS_W && !g->weighted) return fail(WEDGE_ERR_NO_WEIGHTS, "graph has no weights");
            if (which == WEDGE_LAYOUT_XS_W && d.xs_packed)
                return fail(WEDGE_ERR_UNSUPPORTED, "the sliced copy packs the weights into its source words");
            if (which == WEDGE_LAYOUT_XS_SRC) { size = xr * 64 * 4; hsrc = L.xs_src.data(); dsrc = d.xs_src; }
            if (which == WEDGE_LAYOUT_XS_W) { size = xr * 64 * 4; hsrc = L.xs_w.data(); dsrc = d.xs_w; }
            if (which == WEDGE_LAYOUT_XS_ROWMASK) { size = xr * 8; hsrc = L.xs_rowmask.data(); dsrc = d.xs_rowmask; }
            if (which == WEDGE_LAYOUT_XS_ROWSEG) { size = xr * 4; hsrc = L.xs_rowseg.data(); dsrc = d.xs_rowseg; }
            if (which == WEDGE_LAYOUT_XS_NZDST) { size = xseg * 4; hsrc = L.xs_nzdst.data(); dsrc = d.xs_nzdst; }
            if (which == WEDGE_LAYOUT_XS_PR_SPAN_V) { size = d.xs_pspans * 4; hsrc = L.xs_pspan_v.data(); dsrc = d.xs_pspan_v; }
            if (which == WEDGE_LAYOUT_XS_PR_SPAN_OFF) {
                size = d.xs_pspans ? (d.xs_pspans + 1) * 4 : 0;
                hsrc = L.xs_pspan_off.data(); dsrc = d.xs_pspan_off;
            }
            if (which == WEDGE_LAYOUT_XS_PR_SPAN_TILES) { size = d.xs_pspan_pairs * 8; hsrc = L.xs_pspan_tt.data(); dsrc = d.xs_pspan_tt; }
            break;
        }
        case WEDGE_LAYOUT_PERM:
            size = g->perm_host.empty() ? 0 : (uint64_t)d.n * 4;
            if (!size) return fail(WEDGE_ERR_UNSUPPORTED, "graph keeps the caller's ids (no permutation)");
            if (bytes != size) return fail(WEDGE_ERR_INVALID_ARG, "bytes does not match the array size");
            std::memcpy(dst, g->perm_host.data(), size);
            return WEDGE_OK;
        default: return fail(WEDGE_ERR_INVALID_ARG, "unknown layout array");
    }
    if (bytes != size) return fail(WEDGE_ERR_INVALID_ARG, "bytes does not match the array size " + std::to_string(size));
    if (!size) return WEDGE_OK;
    if (g->host_only) { std::memcpy(dst, hsrc, size); return WEDGE_OK; }
    HIP_TRY(hipMemcpy(dst, dsrc, size, hipMemcpyDeviceToHost), "copying layout");
    return WEDGE_OK;
}

wedge_status wedge_bfs(wedge_graph_t g, uint32_t src, uint32_t* level_dev, const wedge_opts* opts,
                       hipStream_t stream, wedge_stats* stats) {
    return debug_verdict(run_frontier_app(kBfs, g, src, level_dev, opts, stream, stats));
}

wedge_status wedge_bfs_noalloc(wedge_graph_t g, uint32_t src, uint32_t* level_dev,
                               const wedge_opts* opts, hipStream_t stream, wedge_stats* stats) {
    return debug_verdict(run_bfs_noalloc(g, src, level_dev, opts, stream, stats));
}

wedge_status wedge_cc(wedge_graph_t g, uint32_t* label_dev, const wedge_opts* opts,
                      hipStream_t stream, wedge_stats* stats) {
    return debug_verdict(run_frontier_app(kCc, g, 0, label_dev, opts, stream, stats));
}

wedge_status wedge_sssp(wedge_graph_t g, uint32_t src, uint32_t* dist_dev, const wedge_opts* opts,
                        hipStream_t stream, wedge_stats* stats) {
    return debug_verdict(run_frontier_app(kSssp, g, src, dist_dev, opts, stream, stats));
}

wedge_status wedge_pagerank(wedge_graph_t g, uint32_t iters, float damping, float* rank_dev,
                            const wedge_opts* opts_in, hipStream_t s, wedge_stats* stats) {
    Range run_range("wedge_pagerank");
    const wedge_opts& o = opts_in ? *opts_in : kDefaultOpts;
    wedge_status st = check_run(g, rank_dev, &o);
    if (st != WEDGE_OK) return st;
    if (!(damping > 0.0f && damping < 1.0f)) return fail(WEDGE_ERR_INVALID_ARG, "damping must be in (0, 1)");
    if (o.flags & (WEDGE_RUN_INPLACE | WEDGE_RUN_PERSISTENT))
        return fail(WEDGE_ERR_UNSUPPORTED, "PageRank runs the synchronous host-driven pull");
    if ((st = check_rows(o, false)) != WEDGE_OK) return st;
    RunGuard guard(g->busy);
    if (!guard.ok) return fail(WEDGE_ERR_BUSY, "graph is in use by another run");
    wedge_stats local{};
    const double t0 = now_ms();
    const DevGraph& d = g->dev;
    if (d.n == 0) { if (stats) *stats = local; return WEDGE_OK; }
    Workspace& w = g->ws;
    if ((st = ensure_workspace(g, 6, false, false)) != WEDGE_OK) return st;
    // each buffer is allocated on its own when missing (see ensure_workspace)
    // tiles of the canonical layout, or of the source-sliced copy when the
    // pull runs over that (its slices start on tile boundaries)
    w.pr_tiles = std::max<uint64_t>((d.rows + kPrTileRows - 1) / kPrTileRows, d.xs_rows / kPrTileRows);
    w.pr_parts = pr_epilogue_blocks(d.n);
    auto need = [&](void** p, size_t bytes, const char* what) -> wedge_status {
        return *p ? WEDGE_OK : dev_alloc(g, p, bytes, what);
    };
    if ((st = need((void**)&w.pr_sum, (size_t)d.n * 4, "PageRank sums")) != WEDGE_OK) return st;
    // slice-major contributions span whole groups of every slice (xs_contrib_cap)
    const uint64_t cap = xs_contrib_cap(d);
    const uint64_t contrib_len = std::max<uint64_t>(d.n, cap << d.xs_lg);
    if ((st = need((void**)&w.pr_contrib, (size_t)contrib_len * 4, "PageRank contributions")) != WEDGE_OK) return st;
    if ((st = need((void**)&w.pr_head, w.pr_tiles * 4, "PageRank tile heads")) != WEDGE_OK) return st;
    if ((st = need((void**)&w.pr_tail, w.pr_tiles * 4, "PageRank tile tails")) != WEDGE_OK) return st;
    if ((st = need((void**)&w.pr_part, (size_t)w.pr_parts * 8, "PageRank partials")) != WEDGE_OK) return st;
    if ((st = need((void**)&w.pr_d, 16, "dangling mass")) != WEDGE_OK) return st;
    if (d.inv && (st = need((void**)&w.pr_rank, (size_t)d.n * 4, "ranks")) != WEDGE_OK) return st;
    float* rank = d.inv ? w.pr_rank : rank_dev;
    const bool time_pull = o.flags & WEDGE_RUN_TIME_PULL;
    const int cus = device_cus(g->device);
    std::vector<hipEvent_t> evs;
    auto cleanup = [&] {
        SetupLock lock;
        for (auto ev : evs) if (ev) (void)hipEventDestroy(ev);
    };
    if (time_pull) {
        SetupLock lock;
        evs.assign(2 * (size_t)iters, nullptr);
        for (auto& ev : evs) {
            const hipError_t ce = hipEventCreate(&ev);
            if (ce != hipSuccess) { ev = nullptr; cleanup(); return hip_fail(ce, "event"); }
        }
    }
    // D_0 comes from the host; D_k (k >= 1) is reduced from the previous
    // epilogue's partials by the fix-up launch of iteration k
    hipError_t e = launch_pr_init(d.n, d.row_off, rank, w.pr_contrib, w.pr_sum, s, d.xs_lg, cap);
    if (e == hipSuccess) e = launch_set_f64(w.pr_d, (double)g->dangling / (double)d.n, s);
    for (uint32_t k = 0; k < iters && e == hipSuccess; ++k) {
        double* dk = w.pr_d + (k & 1);
        if (time_pull) e = hipEventRecord(evs[2 * k], s);
        if (e == hipSuccess) e = launch_pr_pull(d, w.pr_contrib, w.pr_sum, w.pr_head, w.pr_tail, cus, s);
        if (time_pull && e == hipSuccess) e = hipEventRecord(evs[2 * k + 1], s);
        if (e == hipSuccess)
            e = launch_pr_fixup(d, w.pr_head, w.pr_tail, w.pr_sum, w.pr_part, w.pr_parts,
                                k ? dk : nullptr, s);
        if (e == hipSuccess)
            e = launch_pr_epilogue(d.n, d.row_off, w.pr_sum, (double)damping, dk, rank,
                                   w.pr_contrib, w.pr_part, w.pr_parts, s, d.xs_lg, cap);
    }
    if (e == hipSuccess && d.inv) e = launch_unpermute_f32(d.n, d.perm, rank, rank_dev, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "PageRank"); }
    for (uint32_t k = 0; k < iters && time_pull; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, evs[2 * k], evs[2 * k + 1]) == hipSuccess) local.pull_ms += ms;
    }
    cleanup();
    local.iterations = iters;
    local.full_iters = iters;
    local.pull_launches = iters;
    local.full_pull_ms = local.pull_ms;
    local.full_pull_launches = iters;
    local.edges_scanned = (uint64_t)iters * d.m;
    local.ms = now_ms() - t0;
    if (stats) *stats = local;
    return WEDGE_OK;
}

wedge_status wedge_frontier_translate(wedge_graph_t g, const uint32_t* frontier_dev,
                                      uint32_t count, uint32_t chunk_edges, uint64_t* wbits_dev,
                                      uint32_t* chunk_list_dev, uint64_t* marked,
                                      hipStream_t s) {
    if (!g || !marked || !wbits_dev || !chunk_list_dev || (count && !frontier_dev))
        return fail(WEDGE_ERR_INVALID_ARG, "null argument");
    if (g->host_only) return fail(WEDGE_ERR_UNSUPPORTED, "graph was created with WEDGE_HOST_ONLY");
    if (!is_pow2(chunk_edges) || chunk_edges > 4096)
        return fail(WEDGE_ERR_INVALID_ARG, "chunk_edges must be a power of two in [1, 4096]");
    const DevGraph& d = g->dev;
    if (count > d.n) return fail(WEDGE_ERR_INVALID_ARG, "count exceeds n");
    RunGuard guard(g->busy);
    if (!guard.ok) return fail(WEDGE_ERR_BUSY, "graph is in use by another run");
    const int lc = log2u(chunk_edges);
    const uint64_t nchunks = (d.m + chunk_edges - 1) >> lc;
    const uint64_t words = (nchunks + 63) / 64;
    wedge_status st = ensure_workspace(g, lc, true, false);
    if (st != WEDGE_OK) return st;
    Workspace& w = g->ws;
    // the caller's list gets its out-degree prefix through the frontier bitmap
    // (ids are checked on the device: out-of-range ids are ignored)
    HIP_TRY(hipMemsetAsync(w.fbits, 0, ((uint64_t)d.n + 63) / 64 * 8, s), "clearing frontier bitmap");
    HIP_TRY(hipMemsetAsync(w.ctl, 0, sizeof(Ctl), s), "clearing counters");
    HIP_TRY(hipMemsetAsync(wbits_dev, 0, words * 8, s), "clearing caller bitmap");
    std::vector<uint32_t> ids(count);
    if (count) {
        HIP_TRY(hipMemcpyAsync(ids.data(), frontier_dev, (size_t)count * 4, hipMemcpyDeviceToHost, s), "reading frontier");
        HIP_TRY(hipStreamSynchronize(s), "reading frontier");
        for (uint32_t i = 0; i < count; ++i)
            if (ids[i] >= d.n) return fail(WEDGE_ERR_INVALID_ARG, "frontier vertex out of range");
        // set the bits on the host side copy, upload, and let the compaction
        // build the list and the out-degree prefix exactly as an iteration does
        std::vector<uint64_t> fb(((uint64_t)d.n + 63) / 64, 0);
        for (uint32_t v : ids) {
            if (!g->perm_host.empty()) v = g->perm_host[v];
            fb[v >> 6] |= 1ull << (v & 63);
        }
        HIP_TRY(hipMemcpyAsync(w.fbits, fb.data(), fb.size() * 8, hipMemcpyHostToDevice, s), "uploading frontier");
        HIP_TRY(launch_fill_u32_kernel(w.fsum, sum_flags(d.n), 1u, s), "marking frontier summary");
        HIP_TRY(launch_finalize(w.fbits, d.n, d.row_off, w.flist[0], w.degpre[0], w.ctl, nullptr, nullptr,
                                nullptr, w.fsum, nullptr, s), "frontier list");
        HIP_TRY(hipMemcpyAsync(w.ctl_host, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s), "reading counters");
        HIP_TRY(hipStreamSynchronize(s), "frontier list");
        const uint64_t flisted = w.ctl_host->fnext >> kDegBits;
        const uint64_t active = w.ctl_host->fnext & kDegMask;
        HIP_TRY(hipMemsetAsync(w.ctl, 0, sizeof(Ctl), s), "clearing counters");
        HIP_TRY(launch_translate(w.flist[0], w.degpre[0], (uint32_t)flisted, active, d.row_off, d.pos,
                                 lc, wbits_dev, nullptr, s), "frontier translation");
    }
    // compact a copy so the caller keeps the bitmap
    uint64_t* tmp = nullptr;
    SetupLock scratch_lock;
    HIP_TRY(hipMallocAsync((void**)&tmp, words ? words * 8 : 8, s), "scratch bitmap");
    hipError_t e = hipMemcpyAsync(tmp, wbits_dev, words * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_compact_chunks(tmp, words, chunk_list_dev, w.ctl, nullptr, s);
    const hipError_t fe = hipFreeAsync(tmp, s);
    if (e != hipSuccess) return hip_fail(e, "chunk compaction");
    HIP_TRY(fe, "scratch bitmap");
    HIP_TRY(hipMemcpyAsync(w.ctl_host, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s), "reading counters");
    HIP_TRY(hipStreamSynchronize(s), "frontier translation");
    *marked = w.ctl_host->marked >> kDegBits;
    return WEDGE_OK;
}

wedge_status wedge_bfs_multisource(wedge_graph_t g, const uint32_t* srcs, uint32_t count,
                                   uint32_t* levels_dev, const wedge_opts* opts,
                                   hipStream_t stream, wedge_stats* stats) {
    return debug_verdict(run_multisource(g, srcs, count, levels_dev, opts, stream, stats));
}

wedge_status wedge_graph_create_batch_csr(uint32_t count, const uint32_t* n_each,
                                          const uint64_t* const* row_off,
                                          const uint32_t* const* col, uint32_t flags,
                                          hipStream_t stream, wedge_graph_t* out) {
    if (!out) return fail(WEDGE_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!count || !n_each || !row_off || !col) return fail(WEDGE_ERR_INVALID_ARG, "null argument or empty batch");
    if (flags & WEDGE_INPUT_DEVICE) return fail(WEDGE_ERR_INVALID_ARG, "batch parts must be host arrays");
    try {
        std::vector<uint64_t> first(count + 1, 0);
        uint64_t m = 0;
        for (uint32_t i = 0; i < count; ++i) {
            if (!row_off[i]) return fail(WEDGE_ERR_INVALID_ARG, "part offsets pointer is null");
            first[i + 1] = first[i] + n_each[i];
            m += row_off[i][n_each[i]];
        }
        if (first[count] >= (1ull << 31)) return fail(WEDGE_ERR_BAD_GRAPH, "batch has >= 2^31 vertices");
        if (m >= (1ull << 32)) return fail(WEDGE_ERR_BAD_GRAPH, "batch has >= 2^32 edges");
        const uint32_t n = (uint32_t)first[count];
        std::vector<uint64_t> ro((size_t)n + 1, 0);
        std::vector<uint32_t> cl(m ? m : 1);
        uint64_t e = 0;
        for (uint32_t i = 0; i < count; ++i) {
            const uint64_t* r = row_off[i];
            const uint32_t ni = n_each[i];
            if (r[0] != 0) return fail(WEDGE_ERR_BAD_GRAPH, "part offsets must start at 0");
            if (r[ni] && !col[i]) return fail(WEDGE_ERR_INVALID_ARG, "part edge array pointer is null");
            for (uint32_t v = 0; v < ni; ++v) {
                if (r[v + 1] < r[v]) return fail(WEDGE_ERR_BAD_GRAPH, "part offsets are not non-decreasing");
                ro[first[i] + v + 1] = e + r[v + 1];
            }
            for (uint64_t j = 0; j < r[ni]; ++j) {
                if (col[i][j] >= ni) return fail(WEDGE_ERR_BAD_GRAPH, "part neighbour id out of range");
                cl[e + j] = (uint32_t)first[i] + col[i][j];
            }
            e += r[ni];
        }
        wedge_status st = create(true, n, m, ro.data(), cl.data(), nullptr, flags, stream, out);
        if (st != WEDGE_OK) return st;
        (*out)->parts = first;
        return WEDGE_OK;
    } catch (const std::bad_alloc&) {
        return fail(WEDGE_ERR_OOM, "host allocation failed while building the batch");
    }
}

wedge_status wedge_graph_batch_parts(wedge_graph_t g, uint64_t* first, uint32_t cap,
                                     uint32_t* count) {
    if (!g || !count) return fail(WEDGE_ERR_INVALID_ARG, "null argument");
    if (g->parts.empty()) return fail(WEDGE_ERR_UNSUPPORTED, "not a batch graph");
    *count = (uint32_t)g->parts.size() - 1;
    if (first) {
        if (cap < g->parts.size()) return fail(WEDGE_ERR_INVALID_ARG, "cap must be at least count + 1");
        std::memcpy(first, g->parts.data(), g->parts.size() * sizeof(uint64_t));
    }
    return WEDGE_OK;
}

wedge_status wedge_bfs_batch(wedge_graph_t g, const uint32_t* srcs, uint32_t* levels_dev,
                             const wedge_opts* opts, hipStream_t stream, wedge_stats* stats) {
    if (!g) return fail(WEDGE_ERR_INVALID_ARG, "graph is null");
    if (g->parts.empty()) return fail(WEDGE_ERR_UNSUPPORTED, "not a batch graph (wedge_graph_create_batch_csr)");
    if (!srcs) return fail(WEDGE_ERR_INVALID_ARG, "sources pointer is null");
    const uint32_t count = (uint32_t)g->parts.size() - 1;
    std::vector<uint32_t> roots(count);
    for (uint32_t i = 0; i < count; ++i) {
        if ((uint64_t)srcs[i] >= g->parts[i + 1] - g->parts[i])
            return fail(WEDGE_ERR_INVALID_ARG, "source out of range in part " + std::to_string(i));
        roots[i] = (uint32_t)(g->parts[i] + srcs[i]);
    }
    return debug_verdict(run_bfs_roots(g, roots.data(), count, levels_dev, opts, stream, stats));
}

wedge_status wedge_trace_counterfactual(wedge_graph_t g, uint32_t app, uint32_t src,
                                        const wedge_opts* opts_in, wedge_trace_sample* out,
                                        uint32_t cap, uint32_t* count, hipStream_t s) {
    if (!count || (cap && !out)) return fail(WEDGE_ERR_INVALID_ARG, "null argument");
    *count = 0;
    const wedge_opts& o0 = opts_in ? *opts_in : kDefaultOpts;
    if (app < WEDGE_APP_BFS || app > WEDGE_APP_SSSP) return fail(WEDGE_ERR_INVALID_ARG, "unknown app");
    {
        const wedge_status rs = check_rows(o0, false);
        if (rs != WEDGE_OK) return rs;
    }
    wedge_opts o = o0;
    o.gate = WEDGE_GATE_THRESHOLD;
    o.flags = 0;
    o.trace = nullptr;
    o.trace_cap = 0;
    if (!g) return fail(WEDGE_ERR_INVALID_ARG, "graph is null");
    if (g->host_only) return fail(WEDGE_ERR_UNSUPPORTED, "graph was created with WEDGE_HOST_ONLY");
    const DevGraph& d = g->dev;
    if (app != kCc && src >= d.n) return fail(WEDGE_ERR_INVALID_ARG, "source vertex out of range");
    if (app == kSssp && !g->weighted) return fail(WEDGE_ERR_NO_WEIGHTS, "SSSP needs weights");
    if (app == kCc && !(g->flags & WEDGE_SYMMETRIZE)) return fail(WEDGE_ERR_UNSUPPORTED, "CC needs WEDGE_SYMMETRIZE");
    RunGuard guard(g->busy);
    if (!guard.ok) return fail(WEDGE_ERR_BUSY, "graph is in use by another run");
    if (d.n == 0) return WEDGE_OK;
    const uint32_t def_chunk = app == kBfs ? 32u : 16u;
    const LoopCfg c = loop_cfg(o, d, (App)app, default_theta_ppm(app), def_chunk);
    wedge_status st;
    if ((st = ensure_workspace(g, 4, true, true)) != WEDGE_OK) return st;
    Workspace& w = g->ws;
    LoopCfg c16 = c;
    c16.lc = 4;
    if ((st = clear_bitmaps(g, c16, s)) != WEDGE_OK) return st;
    const uint64_t fwords = ((uint64_t)d.n + 63) / 64;
    struct Tmp {
        void* p = nullptr;
        ~Tmp() {
            if (!p) return;
            SetupLock lock;
            (void)hipFree(p);
        }
    } tval, sv, sp, sf, sc;
    uint32_t* val = d.inv ? w.val : nullptr;
    {
        SetupLock lock;
        if (!val) { HIP_TRY(hipMalloc(&tval.p, (size_t)d.n * 4), "trace values"); val = (uint32_t*)tval.p; }
        HIP_TRY(hipMalloc(&sv.p, (size_t)d.n * 4), "snapshot");
        HIP_TRY(hipMalloc(&sp.p, (size_t)d.n * 4), "snapshot");
        HIP_TRY(hipMalloc(&sf.p, fwords * 8), "snapshot");
        HIP_TRY(hipMalloc(&sc.p, sum_flags(d.n) * 4), "snapshot");
    }
    uint32_t* vprev = app == kBfs ? nullptr : w.val_prev;
    const uint32_t isrc = (app != kCc && !g->perm_host.empty()) ? g->perm_host[src] : src;
    HIP_TRY(hipMemsetAsync(w.ctl, 0, sizeof(Ctl), s), "clearing counters");
    if (app == kCc) {
        HIP_TRY(launch_seed_all(d.n, d.m, d.row_off, d.inv, val, w.val_prev, w.flist[0], w.degpre[0],
                                w.fcur, w.csum, w.ctl, s), "seeding CC");
    } else {
        HIP_TRY(launch_fill_u32(val, d.n, kInf, s), "initialising values");
        if (vprev) HIP_TRY(launch_fill_u32(vprev, d.n, kInf, s), "initialising values");
        HIP_TRY(launch_seed_source(isrc, d.row_off, val, vprev, w.flist[0], w.degpre[0], w.fcur, w.csum, w.ctl, s),
                "seeding source");
    }
    HIP_TRY(hipMemcpyAsync(w.ctl_host, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s), "reading counters");
    HIP_TRY(hipStreamSynchronize(s), "initialising trace");
    uint64_t fcount = w.ctl_host->ftotal, flisted = w.ctl_host->fnext >> kDegBits;
    uint64_t active = w.ctl_host->fnext & kDegMask;
    const uint32_t def_mode = def_chunk == 16 ? 1u : def_chunk == 32 ? 2u : 3u;
    uint32_t prev_mode = 0;
    float prev_us = 0.f;
    int cur = 0;
    for (uint32_t k = 0; fcount > 0; ++k) {
        if (k >= c.max_iters) return fail(WEDGE_ERR_NOT_CONVERGED, "max_iters reached");
        const uint32_t tmode = active < c.thr ? def_mode : 0u;
        HIP_TRY(hipMemcpyAsync(sv.p, val, (size_t)d.n * 4, hipMemcpyDeviceToDevice, s), "snapshot");
        if (vprev) HIP_TRY(hipMemcpyAsync(sp.p, vprev, (size_t)d.n * 4, hipMemcpyDeviceToDevice, s), "snapshot");
        HIP_TRY(hipMemcpyAsync(sf.p, w.fcur, fwords * 8, hipMemcpyDeviceToDevice, s), "snapshot");
        HIP_TRY(hipMemcpyAsync(sc.p, w.csum, sum_flags(d.n) * 4, hipMemcpyDeviceToDevice, s), "snapshot");
        float t[4] = {0, 0, 0, 0};
        for (uint32_t mi = 0; mi < 4; ++mi) {
            if (mi) {
                HIP_TRY(hipMemcpyAsync(val, sv.p, (size_t)d.n * 4, hipMemcpyDeviceToDevice, s), "restore");
                if (vprev) HIP_TRY(hipMemcpyAsync(vprev, sp.p, (size_t)d.n * 4, hipMemcpyDeviceToDevice, s), "restore");
                HIP_TRY(hipMemcpyAsync(w.fcur, sf.p, fwords * 8, hipMemcpyDeviceToDevice, s), "restore");
                HIP_TRY(hipMemcpyAsync(w.csum, sc.p, sum_flags(d.n) * 4, hipMemcpyDeviceToDevice, s), "restore");
            }
            HIP_TRY(hipMemsetAsync(w.ctl, 0, 24, s), "clearing counters");
            HIP_TRY(hipEventRecord(w.ev[0], s), "event");
            if (mi == 0) {
                HIP_TRY(launch_pull_full(app, d, k, val, vprev, w.fcur, w.fbits, w.fsum, s), "full pull");
            } else {
                const int lc = 3 + (int)mi;
                const uint64_t nch = c.chunks_of(lc);
                HIP_TRY(launch_translate(w.flist[cur], w.degpre[cur], (uint32_t)flisted, active, d.row_off,
                                         d.pos, lc, w.wbits, w.wsum, s), "frontier translation");
                HIP_TRY(launch_compact_chunks(w.wbits, (nch + 63) / 64, w.chunks, w.ctl, w.wsum, s), "chunk compaction");
                HIP_TRY(launch_pull_chunks(app, d, k, lc, w.chunks, w.ctl, active < nch ? active : nch, val,
                                           vprev, w.fcur, w.fbits, w.fsum, s), "chunk pull");
            }
            HIP_TRY(launch_finalize(w.fbits, d.n, d.row_off, w.flist[cur ^ 1], w.degpre[cur ^ 1], w.ctl,
                                    vprev, val, w.fcur, w.fsum, w.csum, s, mi == 0, k + 1),
                    "frontier finalisation");
            HIP_TRY(hipEventRecord(w.ev[1], s), "event");
            HIP_TRY(hipEventSynchronize(w.ev[1]), "trace iteration");
            HIP_TRY(hipEventElapsedTime(&t[mi], w.ev[0], w.ev[1]), "event time");
            t[mi] *= 1000.f;
        }
        HIP_TRY(hipMemcpyAsync(w.ctl_host, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s), "reading counters");
        HIP_TRY(hipStreamSynchronize(s), "trace iteration");
        if (*count < cap) {
            wedge_trace_sample& r = out[(*count)++];
            r.app = app;
            r.iter = k;
            r.prev_mode = prev_mode;
            r.threshold_mode = tmode;
            r.n = d.n;
            r.m = d.m;
            r.frontier = fcount;
            r.active = active;
            r.prev_us = prev_us;
            for (int j = 0; j < 4; ++j) r.t_us[j] = t[j];
            r.reserved = 0.f;
        }
        prev_mode = tmode;
        prev_us = t[tmode];
        fcount = w.ctl_host->ftotal;
        flisted = w.ctl_host->fnext >> kDegBits;
        active = w.ctl_host->fnext & kDegMask;
        cur ^= 1;
    }
    return WEDGE_OK;
}

namespace {
// The tuner's table: (kind, source count, ceil(log2 m), compute units) -> the
// winning options. With WEDGE_TUNE_CACHE set, the table also lives in that
// text file: it is read once per process on first use, and rewritten (to a
// temporary file, then renamed) after every tuning run, so tuned choices
// survive the process. Lines: "kind count bucket cus chunk persistent bpc rows"
// after a "wedge-tune-v1" header; malformed lines are ignored.
using TuneKey = std::tuple<uint32_t, uint32_t, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, wedge_opts> g_tune;
bool g_tune_loaded = false;

int size_bucket(uint64_t m) { int b = 0; while ((1ull << b) < m) ++b; return b; }

int current_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { (void)hipGetLastError(); return 0; }
    return device_cus(dev);
}

void tune_cache_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("WEDGE_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    if (!std::fgets(line, sizeof line, f) || std::strncmp(line, "wedge-tune-v1", 13) != 0) {
        std::fclose(f);
        return;
    }
    while (std::fgets(line, sizeof line, f)) {
        unsigned kind, count, chunk, pers, bpc, rows;
        int bucket, cus;
        if (std::sscanf(line, "%u %u %d %d %u %u %u %u", &kind, &count, &bucket, &cus, &chunk, &pers,
                        &bpc, &rows) != 8)
            continue;
        if (kind > WEDGE_TUNE_BATCH || !is_pow2(chunk) || chunk > 4096 || pers > 1 ||
            (rows && rows != 4 && rows != 8 && rows != 16))
            continue;
        wedge_opts o = kDefaultOpts;
        o.chunk_edges = chunk;
        o.flags = pers ? WEDGE_RUN_PERSISTENT : 0u;
        o.blocks_per_cu = bpc;
        o.rows_per_wave = rows;
        g_tune[TuneKey(kind, count, bucket, cus)] = o;
    }
    std::fclose(f);
}

void tune_cache_save_locked() {
    const char* path = std::getenv("WEDGE_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "wedge-tune-v1\n");
    for (const auto& kv : g_tune)
        std::fprintf(f, "%u %u %d %d %u %u %u %u\n", std::get<0>(kv.first), std::get<1>(kv.first),
                     std::get<2>(kv.first), std::get<3>(kv.first), kv.second.chunk_edges,
                     (kv.second.flags & WEDGE_RUN_PERSISTENT) ? 1u : 0u, kv.second.blocks_per_cu,
                     kv.second.rows_per_wave);
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), path);
    else std::remove(tmp.c_str());
}
}  // namespace

wedge_status wedge_tune_bfs(wedge_graph_t g, uint32_t kind, const uint32_t* srcs, uint32_t count,
                            uint32_t* out_dev, hipStream_t stream, wedge_opts* best,
                            double* best_ms) {
    if (!g || !srcs || !out_dev || !best) return fail(WEDGE_ERR_INVALID_ARG, "null argument");
    if (kind > WEDGE_TUNE_BATCH) return fail(WEDGE_ERR_INVALID_ARG, "unknown kind");
    const wedge_opts base = *best;
    struct Cand { uint32_t chunk, persistent, bpc, rows; };
    // host-driven: every pull shape; persistent: per-CU block counts below the
    // occupancy maximum, and the maximum (0). The learned gate runs host-driven.
    int bpc_max = 0;
    if (persistent_max_blocks(kind == WEDGE_TUNE_MULTISOURCE, &bpc_max) != hipSuccess) {
        (void)hipGetLastError();
        bpc_max = 0;
    }
    const bool persistent_ok = base.gate != WEDGE_GATE_LEARNED;
    std::vector<Cand> cands;
    for (uint32_t c : {16u, 32u, 64u}) {
        for (uint32_t r : {4u, 8u, 16u}) cands.push_back({c, 0, 0, r});
        if (!persistent_ok) continue;
        for (uint32_t b : {1u, 2u, 4u})
            if ((int)b < bpc_max) cands.push_back({c, 1, b, 0});
        cands.push_back({c, 1, 0, 0});
    }
    double best_t = 1e300;
    wedge_opts win = base;
    for (const Cand& cd : cands) {
        wedge_opts o = base;
        o.chunk_edges = cd.chunk;
        o.flags = (base.flags & ~(WEDGE_RUN_PERSISTENT | WEDGE_RUN_TIME_ITERS | WEDGE_RUN_TIME_PULL)) |
                  (cd.persistent ? WEDGE_RUN_PERSISTENT : 0u);
        o.blocks_per_cu = cd.bpc;
        o.rows_per_wave = cd.rows;
        o.trace = nullptr;
        o.trace_cap = 0;
        double t = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            wedge_stats st{};
            wedge_status r;
            if (kind == WEDGE_TUNE_SINGLE) r = wedge_bfs(g, srcs[0], out_dev, &o, stream, &st);
            else if (kind == WEDGE_TUNE_MULTISOURCE) r = wedge_bfs_multisource(g, srcs, count, out_dev, &o, stream, &st);
            else r = wedge_bfs_batch(g, srcs, out_dev, &o, stream, &st);
            if (r != WEDGE_OK) return r;
            t = std::min(t, st.ms);
        }
        if (t < best_t) { best_t = t; win = o; }
    }
    *best = win;
    if (best_ms) *best_ms = best_t;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load_locked();
    g_tune[TuneKey(kind, count, size_bucket(g->dev.m), device_cus(g->device))] = win;
    tune_cache_save_locked();
    return WEDGE_OK;
}

wedge_status wedge_tune_lookup(uint32_t kind, uint32_t count, uint64_t m, wedge_opts* opts) {
    if (!opts) return fail(WEDGE_ERR_INVALID_ARG, "null argument");
    const int cus = current_cus();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load_locked();
    auto it = g_tune.find(TuneKey(kind, count, size_bucket(m), cus));
    if (it == g_tune.end()) return fail(WEDGE_ERR_UNSUPPORTED, "no tuned entry for this kind and size");
    opts->chunk_edges = it->second.chunk_edges;
    opts->flags = (opts->flags & ~WEDGE_RUN_PERSISTENT) | (it->second.flags & WEDGE_RUN_PERSISTENT);
    opts->blocks_per_cu = it->second.blocks_per_cu;
    opts->rows_per_wave = it->second.rows_per_wave;
    return WEDGE_OK;
}

const char* wedge_status_string(wedge_status s) {
    switch (s) {
        case WEDGE_OK: return "ok";
        case WEDGE_ERR_INVALID_ARG: return "invalid argument";
        case WEDGE_ERR_BAD_GRAPH: return "malformed graph";
        case WEDGE_ERR_NO_WEIGHTS: return "graph has no weights";
        case WEDGE_ERR_OOM: return "out of memory";
        case WEDGE_ERR_HIP: return "HIP runtime error";
        case WEDGE_ERR_UNSUPPORTED: return "unsupported for this graph";
        case WEDGE_ERR_MODEL: return "invalid model";
        case WEDGE_ERR_NOT_CONVERGED: return "did not converge within max_iters";
        case WEDGE_ERR_BUSY: return "graph busy";
    }
    return "unknown status";
}

const char* wedge_last_error(void) { return g_err.c_str(); }

const char* wedge_version(void) { return "0.1.0"; }

}  // extern "C"
