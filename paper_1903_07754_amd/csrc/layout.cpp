// Host-side construction of the device graph layout (one-off, at graph create).
//
// From the caller's out-edges (CSR) it builds:
//   * the in-edge array (CSC; Background, Graph Representation) with each
//     destination's in-edges ordered by ascending source, weights aligned;
//   * the edge index of the Wedge Frontier (Implementation, Data Structures):
//     pos[q] = in-edge position of CSR edge q, kept in CSR order so that one
//     vertex's entries are contiguous and ascend (out-neighbours ascend, and
//     in-edge positions are grouped by destination);
//   * the row layout the pull kernels use instead of the vertex index: for
//     every 64 consecutive in-edge positions a 64-bit mask of where a
//     destination's in-edge list starts, the segment index covering the row's
//     first position, and the ids of destinations with in-edges. With one wave
//     lane per position, a lane finds its destination with one popcount.
//   * the PageRank tile spans: destinations whose in-edges cross a boundary
//     between pull tiles of kPrTileRows rows.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "wedge_internal.h"

namespace wedge {
namespace {

unsigned host_threads() {
    const char* e = std::getenv("WEDGE_HOST_THREADS");
    if (!e) e = std::getenv("OMP_NUM_THREADS");
    long t = e ? std::strtol(e, nullptr, 10) : 0;
    if (t <= 0) t = (long)std::thread::hardware_concurrency();
    if (t <= 0) t = 1;
    return (unsigned)std::min<long>(t, 64);
}

// Run f(begin, end) over [0, count) split into equal static ranges.
template <class F>
void parallel_ranges(uint64_t count, F&& f) {
    unsigned t = host_threads();
    if (count < 65536 || t == 1) {
        f(0, count);
        return;
    }
    std::vector<std::thread> pool;
    uint64_t step = (count + t - 1) / t;
    for (unsigned i = 0; i < t; ++i) {
        uint64_t b = i * step, e = std::min<uint64_t>(count, b + step);
        if (b >= e) break;
        pool.emplace_back([=, &f] { f(b, e); });
    }
    for (auto& th : pool) th.join();
}

// Run f(i) for i in [0, count) with dynamic chunks (for skewed work).
template <class F>
void parallel_dynamic(uint64_t count, uint64_t grain, F&& f) {
    unsigned t = host_threads();
    if (count < 4096 || t == 1) {
        for (uint64_t i = 0; i < count; ++i) f(i);
        return;
    }
    std::atomic<uint64_t> next{0};
    std::vector<std::thread> pool;
    for (unsigned i = 0; i < t; ++i)
        pool.emplace_back([&] {
            for (;;) {
                uint64_t b = next.fetch_add(grain);
                if (b >= count) break;
                uint64_t e = std::min(count, b + grain);
                for (uint64_t j = b; j < e; ++j) f(j);
            }
        });
    for (auto& th : pool) th.join();
}

wedge_status check_offsets(uint32_t n, uint64_t m, const uint64_t* off, const uint32_t* ids,
                           std::string* err) {
    if (n >= (1u << 31)) { *err = "n must be < 2^31"; return WEDGE_ERR_BAD_GRAPH; }
    if (m >= (1ull << 32)) { *err = "m must be < 2^32 (in-edge positions are 32-bit)"; return WEDGE_ERR_BAD_GRAPH; }
    if (!off) { *err = "offsets pointer is null"; return WEDGE_ERR_INVALID_ARG; }
    if (m && !ids) { *err = "edge array pointer is null"; return WEDGE_ERR_INVALID_ARG; }
    if (off[0] != 0) { *err = "offsets[0] must be 0"; return WEDGE_ERR_BAD_GRAPH; }
    for (uint32_t v = 0; v < n; ++v)
        if (off[v + 1] < off[v]) { *err = "offsets are not non-decreasing at vertex " + std::to_string(v); return WEDGE_ERR_BAD_GRAPH; }
    if (off[n] != m) { *err = "offsets[n] != m"; return WEDGE_ERR_BAD_GRAPH; }
    std::atomic<uint64_t> bad{~0ull};
    parallel_ranges(m, [&](uint64_t b, uint64_t e) {
        for (uint64_t j = b; j < e; ++j)
            if (ids[j] >= n) { bad.store(j); break; }
    });
    if (bad.load() != ~0ull) {
        *err = "vertex id out of range at edge " + std::to_string(bad.load());
        return WEDGE_ERR_BAD_GRAPH;
    }
    return WEDGE_OK;
}

// Undirected view of a CSR: both directions of every non-loop edge, merged.
void symmetrize_csr(uint32_t n, const uint64_t* row_off, const uint32_t* col,
                    std::vector<uint64_t>* sro, std::vector<uint32_t>* scol) {
    std::vector<uint64_t> deg((size_t)n + 1, 0);
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t j = row_off[u]; j < row_off[u + 1]; ++j)
            if (col[j] != u) { deg[u + 1]++; deg[col[j] + 1]++; }
    for (uint32_t v = 0; v < n; ++v) deg[v + 1] += deg[v];
    std::vector<uint32_t> tmp(deg[n] ? deg[n] : 1);
    std::vector<uint64_t> cur(deg.begin(), deg.end());
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t j = row_off[u]; j < row_off[u + 1]; ++j)
            if (col[j] != u) { tmp[cur[u]++] = col[j]; tmp[cur[col[j]]++] = u; }
    std::vector<uint32_t> kept(n, 0);
    parallel_dynamic(n, 1024, [&](uint64_t u) {
        uint32_t* b = tmp.data() + deg[u];
        uint32_t* e = tmp.data() + deg[u + 1];
        std::sort(b, e);
        kept[u] = (uint32_t)(std::unique(b, e) - b);
    });
    sro->assign((size_t)n + 1, 0);
    for (uint32_t u = 0; u < n; ++u) (*sro)[u + 1] = (*sro)[u] + kept[u];
    scol->resize((*sro)[n]);
    parallel_dynamic(n, 1024, [&](uint64_t u) {
        std::memcpy(scol->data() + (*sro)[u], tmp.data() + deg[u], kept[u] * sizeof(uint32_t));
    });
}


// Relabel a CSR so that internal vertex i is the i-th vertex in order of
// decreasing out-degree (ties by id): inv[i] = original id, perm[orig] = i.
// Rows of the result list internal neighbour ids in ascending order (parallel
// edges keep their input order); weights follow their edges.
void relabel_csr(uint32_t n, const uint64_t* row_off, const uint32_t* col, const uint32_t* w,
                 std::vector<uint32_t>* perm, std::vector<uint32_t>* inv,
                 std::vector<uint64_t>* nro, std::vector<uint32_t>* ncol,
                 std::vector<uint32_t>* nw) {
    uint64_t maxdeg = 0;
    for (uint32_t u = 0; u < n; ++u) maxdeg = std::max<uint64_t>(maxdeg, row_off[u + 1] - row_off[u]);
    // counting sort by degree (descending), stable in id
    std::vector<uint64_t> bucket(maxdeg + 2, 0);
    for (uint32_t u = 0; u < n; ++u) bucket[maxdeg - (row_off[u + 1] - row_off[u]) + 1]++;
    for (uint64_t d = 0; d <= maxdeg; ++d) bucket[d + 1] += bucket[d];
    inv->resize(n);
    perm->resize(n);
    for (uint32_t u = 0; u < n; ++u) (*inv)[bucket[maxdeg - (row_off[u + 1] - row_off[u])]++] = u;
    for (uint32_t i = 0; i < n; ++i) (*perm)[(*inv)[i]] = i;
    nro->assign((size_t)n + 1, 0);
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t u = (*inv)[i];
        (*nro)[i + 1] = (*nro)[i] + (row_off[u + 1] - row_off[u]);
    }
    const uint64_t m = (*nro)[n];
    ncol->resize(m ? m : 1);
    if (nw) nw->resize(m ? m : 1);
    const std::vector<uint32_t>& P = *perm;
    parallel_dynamic(n, 1024, [&](uint64_t i) {
        const uint32_t u = (*inv)[i];
        const uint64_t b = row_off[u], d = row_off[u + 1] - b, o = (*nro)[i];
        if (!d) return;
        std::vector<uint64_t> key(d);
        for (uint64_t j = 0; j < d; ++j) key[j] = ((uint64_t)P[col[b + j]] << 32) | j;
        std::sort(key.begin(), key.end());
        for (uint64_t j = 0; j < d; ++j) {
            (*ncol)[o + j] = (uint32_t)(key[j] >> 32);
            if (nw) (*nw)[o + j] = w[b + (uint32_t)key[j]];
        }
    });
}

}  // namespace

wedge_status build_layout_from_csr(uint32_t n, uint64_t m, const uint64_t* row_off_in,
                                   const uint32_t* col_in, const uint32_t* w, bool symmetrize,
                                   bool relabel, HostLayout* L, std::string* err) {
    wedge_status st = check_offsets(n, m, row_off_in, col_in, err);
    if (st != WEDGE_OK) return st;
    std::vector<uint64_t> sro;
    std::vector<uint32_t> scol;
    const uint64_t* row_off = row_off_in;
    const uint32_t* col = col_in;
    if (symmetrize) {
        if (w) { *err = "weights are not accepted with WEDGE_SYMMETRIZE"; return WEDGE_ERR_INVALID_ARG; }
        symmetrize_csr(n, row_off_in, col_in, &sro, &scol);
        row_off = sro.data();
        col = scol.data();
        m = sro[n];
        if (m >= (1ull << 32)) { *err = "undirected view has >= 2^32 edges"; return WEDGE_ERR_BAD_GRAPH; }
    }
    // --- internal vertex order: out-degree descending (ties by id), so the
    // values most often gathered by the pull (sources with many out-edges)
    // share cache lines; the ABI keeps the caller's ids (perm maps them).
    std::vector<uint64_t> rro;
    std::vector<uint32_t> rcol, rw;
    if (relabel && n) {
        relabel_csr(n, row_off, col, w, &L->perm, &L->inv, &rro, &rcol, w ? &rw : nullptr);
        row_off = rro.data();
        col = rcol.data();
        if (w) w = rw.data();
    }
    L->n = n;
    L->m = m;

    // --- in-degrees and in-edge offsets
    std::vector<uint32_t> indeg(n, 0);
    parallel_ranges(m, [&](uint64_t b, uint64_t e) {
        for (uint64_t j = b; j < e; ++j) __atomic_fetch_add(&indeg[col[j]], 1u, __ATOMIC_RELAXED);
    });
    L->col_off.assign((size_t)n + 1, 0);
    for (uint32_t v = 0; v < n; ++v) L->col_off[v + 1] = L->col_off[v] + indeg[v];

    // --- scatter (source << 32 | csr index) into destination buckets, then sort
    // each bucket: sources ascend, duplicate edges keep CSR order
    std::vector<uint64_t> keys(m ? m : 1);
    {
        std::vector<uint32_t> cur(L->col_off.begin(), L->col_off.end() - 1);
        // sources of a range of CSR edges: walk rows
        parallel_ranges(n, [&](uint64_t ub, uint64_t ue) {
            for (uint64_t u = ub; u < ue; ++u)
                for (uint64_t j = row_off[u]; j < row_off[u + 1]; ++j) {
                    uint32_t p = __atomic_fetch_add(&cur[col[j]], 1u, __ATOMIC_RELAXED);
                    keys[p] = (u << 32) | j;
                }
        });
    }
    parallel_dynamic(n, 2048, [&](uint64_t v) {
        uint32_t b = L->col_off[v], e = L->col_off[v + 1];
        if (e - b > 1) std::sort(keys.begin() + b, keys.begin() + e);
    });
    L->in_src.resize(m);
    L->pos.resize(m);
    if (w) L->in_w.resize(m);
    std::atomic<uint32_t> maxw{0};
    parallel_ranges(m, [&](uint64_t b, uint64_t e) {
        uint32_t mw = 0;
        for (uint64_t p = b; p < e; ++p) {
            uint64_t k = keys[p];
            uint32_t q = (uint32_t)k;
            L->in_src[p] = (uint32_t)(k >> 32);
            L->pos[q] = (uint32_t)p;
            if (w) { L->in_w[p] = w[q]; mw = std::max(mw, w[q]); }
        }
        uint32_t old = maxw.load();
        while (mw > old && !maxw.compare_exchange_weak(old, mw)) {}
    });
    L->max_w = maxw.load();
    std::vector<uint64_t>().swap(keys);

    // --- out-edge offsets (32-bit) and dangling count
    L->row_off.resize((size_t)n + 1);
    uint32_t dang = 0;
    for (uint32_t u = 0; u <= n; ++u) L->row_off[u] = (uint32_t)row_off[u];
    for (uint32_t u = 0; u < n; ++u) dang += row_off[u + 1] == row_off[u];
    L->dangling = dang;

    // --- destinations with in-edges, row masks, row segment bases
    L->nzdst.clear();
    L->nzdst.reserve(n);
    for (uint32_t v = 0; v < n; ++v)
        if (indeg[v]) L->nzdst.push_back(v);
    uint64_t rows = (m + 63) / 64;
    L->rowmask.assign(rows, 0);
    L->rowseg.assign(rows, 0);
    uint64_t s = 0;
    const uint64_t S = L->nzdst.size();
    for (uint64_t r = 0; r < rows; ++r) {
        uint64_t lo = r * 64, hi = lo + 64;
        // advance s to the last segment starting at or before lo
        while (s + 1 < S && L->col_off[L->nzdst[s + 1]] <= lo) ++s;
        L->rowseg[r] = (uint32_t)s;
        for (uint64_t t = s; t < S; ++t) {
            uint64_t st0 = L->col_off[L->nzdst[t]];
            if (st0 >= hi) break;
            if (st0 >= lo) L->rowmask[r] |= 1ull << (st0 - lo);
        }
    }

    // --- PageRank tile spans (short ones first, then those over more than
    // kPrShortSpan tiles; each group ordered by vertex)
    L->spans.clear();
    std::vector<uint32_t> longs;
    const uint64_t T = 64ull * kPrTileRows;
    for (uint64_t t = 0; t < S; ++t) {
        uint32_t v = L->nzdst[t];
        uint64_t a = L->col_off[v], b = (uint64_t)L->col_off[v + 1] - 1;
        if (a / T != b / T) {
            std::vector<uint32_t>& dst = (b / T - a / T <= kPrShortSpan) ? L->spans : longs;
            dst.push_back(v);
            dst.push_back((uint32_t)(a / T));
            dst.push_back((uint32_t)(b / T));
        }
    }
    L->short_spans = L->spans.size() / 3;
    L->spans.insert(L->spans.end(), longs.begin(), longs.end());
    return WEDGE_OK;
}

uint32_t xs_slices_lg(uint64_t sources) {
    const char* e = std::getenv("WEDGE_XS_SLICES");
    if (e && *e) {
        const long v = std::strtol(e, nullptr, 10);
        for (uint32_t lg = 3; (1 << lg) <= kMaxSlices; ++lg)
            if (v == (1 << lg)) return lg;
    }
    uint32_t lg = 3;
    while ((1 << lg) < kMaxSlices && sources * 4 > (kSliceValueBytes << lg)) ++lg;
    return lg;
}

void build_xcd_slices(HostLayout* L) {
    const uint32_t n = L->n;
    const bool weighted = !L->in_w.empty();
    // weighted graphs whose weights fit 8 bits and slice-local ids 24 bits
    // store one word per in-edge instead of two
    const bool packed = weighted && L->max_w <= kXsPackMaxW && (uint64_t)n <= kXsPackMaxN;
    L->xs_packed = packed;
    uint64_t sources = 0;
    for (uint32_t v = 0; v < n; ++v) sources += L->row_off[v + 1] > L->row_off[v];
    const uint32_t lg = xs_slices_lg(sources);
    const int S = 1 << lg;
    L->xs_lg = lg;
    // per thread range of destinations: edge counts per slice
    const unsigned T = std::max(1u, std::min<unsigned>(host_threads(), 64));
    const uint64_t step = ((uint64_t)n + T - 1) / T;
    std::vector<uint64_t> cnt((size_t)T * S, 0);
    auto for_ranges = [&](auto&& f) {
        std::vector<std::thread> pool;
        for (unsigned t = 0; t < T; ++t) {
            const uint64_t b = t * step, e = std::min<uint64_t>(n, b + step);
            if (b >= e) break;
            pool.emplace_back([=, &f] { f(t, b, e); });
        }
        for (auto& th : pool) th.join();
    };
    for_ranges([&](unsigned t, uint64_t vb, uint64_t ve) {
        uint64_t* c = &cnt[(size_t)t * S];
        for (uint64_t p = L->col_off[vb]; p < L->col_off[ve]; ++p) c[xcd_slice_of(L->in_src[p], lg)]++;
    });
    // slice starts are aligned to PageRank tiles (kPrTileRows rows), so no tile
    // straddles two slices; inside a slice, thread ranges follow in order
    const uint64_t align = 64ull * kPrTileRows;
    std::vector<uint64_t> base((size_t)T * S, 0);
    uint64_t at = 0;
    for (int j = 0; j < S; ++j) {
        at = (at + align - 1) & ~(align - 1);
        L->xs_row_begin[j] = (uint32_t)(at / 64);
        for (unsigned t = 0; t < T; ++t) {
            base[(size_t)t * S + j] = at;
            at += cnt[(size_t)t * S + j];
        }
        L->xs_edge_end[j] = (uint32_t)at;
    }
    const uint64_t total = (at + align - 1) & ~(align - 1);
    const uint64_t rows = total / 64;
    L->xs_row_begin[S] = (uint32_t)rows;
    L->xs_src.assign(total ? total : 1, 0);
    if (weighted && !packed) L->xs_w.assign(total ? total : 1, 0);
    // destination of every position (padding: none), for the row layout below
    std::vector<uint32_t> dst(total ? total : 1, 0xFFFFFFFFu);
    for_ranges([&](unsigned t, uint64_t vb, uint64_t ve) {
        uint64_t cur[kMaxSlices];
        for (int j = 0; j < S; ++j) cur[j] = base[(size_t)t * S + j];
        // destinations ascend, and each destination's sources ascend, so every
        // slice keeps the canonical (destination, source) order
        for (uint64_t v = vb; v < ve; ++v)
            for (uint64_t p = L->col_off[v]; p < L->col_off[v + 1]; ++p) {
                const uint32_t u = L->in_src[p];
                const uint64_t q = cur[xcd_slice_of(u, lg)]++;
                if (packed) {
                    L->xs_src[q] = (xcd_slice_local(u, lg) << 8) | L->in_w[p];
                } else {
                    L->xs_src[q] = u;
                    if (weighted) L->xs_w[q] = L->in_w[p];
                }
                dst[q] = (uint32_t)v;
            }
    });
    // row layout: a segment starts at a slice's first position and wherever the
    // destination changes; padding positions start nothing
    L->xs_rowmask.assign(rows ? rows : 1, 0);
    std::vector<uint32_t> starts(rows ? rows : 1, 0);
    std::vector<uint8_t> slice_row(rows ? rows : 1, 0);  // rows where a slice starts
    for (int j = 0; j < S; ++j)
        if (L->xs_row_begin[j] < rows) slice_row[L->xs_row_begin[j]] = 1;
    parallel_ranges(rows, [&](uint64_t rb, uint64_t re) {
        for (uint64_t r = rb; r < re; ++r) {
            uint64_t mk = 0;
            for (int l = 0; l < 64; ++l) {
                const uint64_t q = r * 64 + l;
                if (dst[q] == 0xFFFFFFFFu) continue;
                bool start = q == 0 || dst[q - 1] != dst[q];
                if (l == 0 && slice_row[r]) start = true;  // a new slice
                if (start) mk |= 1ull << l;
            }
            L->xs_rowmask[r] = mk;
            starts[r] = (uint32_t)__builtin_popcountll(mk);
        }
    });
    L->xs_rowseg.assign(rows ? rows : 1, 0);
    uint64_t segs = 0;
    for (uint64_t r = 0; r < rows; ++r) {
        // the segment covering the row's first position: the one starting there,
        // else the last one started before it
        L->xs_rowseg[r] = (uint32_t)((L->xs_rowmask[r] & 1ull) ? segs : segs - 1);
        segs += starts[r];
    }
    L->xs_nzdst.resize(segs ? segs : 1);
    std::vector<uint64_t> seg_begin(segs + 1, 0);
    {
        uint64_t sidx = 0;
        for (uint64_t r = 0; r < rows; ++r) {
            uint64_t mk = L->xs_rowmask[r];
            while (mk) {
                const int l = __builtin_ctzll(mk);
                mk &= mk - 1;
                seg_begin[sidx] = r * 64 + l;
                L->xs_nzdst[sidx++] = dst[r * 64 + l];
            }
        }
    }
    L->xs_nzdst.resize(segs);
    // PageRank: segments whose positions cross a tile boundary, grouped by
    // destination (a destination has at most one segment per slice; its
    // crossing segments are listed in slice order). A segment ends at the next
    // segment's start or its slice's end.
    const uint64_t TE = 64ull * kPrTileRows;  // positions per tile
    struct Span { uint32_t v, a, b; };
    std::vector<Span> sp;
    {
        int j = 0;
        for (uint64_t t = 0; t < segs; ++t) {
            const uint64_t a = seg_begin[t];
            while (j + 1 < S && a >= (uint64_t)L->xs_row_begin[j + 1] * 64) ++j;
            uint64_t e = t + 1 < segs ? seg_begin[t + 1] : (uint64_t)L->xs_edge_end[j];
            e = std::min<uint64_t>(e, L->xs_edge_end[j]);
            const uint64_t b = e - 1;
            if (a / TE != b / TE) sp.push_back({L->xs_nzdst[t], (uint32_t)(a / TE), (uint32_t)(b / TE)});
        }
    }
    std::stable_sort(sp.begin(), sp.end(), [](const Span& x, const Span& y) { return x.v < y.v; });
    // per destination: its pairs; short destinations (at most kPrShortSpan
    // extra tiles over all their spans) first, then the long ones
    std::vector<uint32_t> sv, sl, lv, ll;  // vertex, first pair index
    std::vector<uint32_t> pairs_short, pairs_long;
    for (size_t i = 0; i < sp.size();) {
        size_t k = i;
        uint64_t extra = 0;
        while (k < sp.size() && sp[k].v == sp[i].v) { extra += sp[k].b - sp[k].a; ++k; }
        const bool is_short = extra <= kPrShortSpan;
        std::vector<uint32_t>& vv = is_short ? sv : lv;
        std::vector<uint32_t>& off = is_short ? sl : ll;
        std::vector<uint32_t>& pr = is_short ? pairs_short : pairs_long;
        vv.push_back(sp[i].v);
        off.push_back((uint32_t)(pr.size() / 2));
        for (size_t q = i; q < k; ++q) { pr.push_back(sp[q].a); pr.push_back(sp[q].b); }
        i = k;
    }
    L->xs_pspan_short = sv.size();
    L->xs_pspan_v = sv;
    L->xs_pspan_v.insert(L->xs_pspan_v.end(), lv.begin(), lv.end());
    const uint32_t npairs_short = (uint32_t)(pairs_short.size() / 2);
    L->xs_pspan_off = sl;
    for (uint32_t o : ll) L->xs_pspan_off.push_back(o + npairs_short);
    L->xs_pspan_off.push_back((uint32_t)((pairs_short.size() + pairs_long.size()) / 2));
    L->xs_pspan_tt = pairs_short;
    L->xs_pspan_tt.insert(L->xs_pspan_tt.end(), pairs_long.begin(), pairs_long.end());
}

wedge_status build_layout_from_csc(uint32_t n, uint64_t m, const uint64_t* col_off,
                                   const uint32_t* src, const uint32_t* w, bool symmetrize,
                                   bool relabel, HostLayout* L, std::string* err) {
    wedge_status st = check_offsets(n, m, col_off, src, err);
    if (st != WEDGE_OK) return st;
    // transpose to CSR (stable: destinations ascend within each source's row)
    std::vector<uint64_t> row_off((size_t)n + 1, 0);
    for (uint64_t p = 0; p < m; ++p) row_off[src[p] + 1]++;
    for (uint32_t u = 0; u < n; ++u) row_off[u + 1] += row_off[u];
    std::vector<uint64_t> cur(row_off.begin(), row_off.end() - 1);
    std::vector<uint32_t> col(m ? m : 1);
    std::vector<uint32_t> cw(w ? (m ? m : 1) : 0);
    for (uint32_t v = 0; v < n; ++v)
        for (uint64_t p = col_off[v]; p < col_off[v + 1]; ++p) {
            uint64_t q = cur[src[p]]++;
            col[q] = v;
            if (w) cw[q] = w[p];
        }
    return build_layout_from_csr(n, m, row_off.data(), col.data(), w ? cw.data() : nullptr,
                                 symmetrize, relabel, L, err);
}

}  // namespace wedge
