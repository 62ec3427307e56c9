// HIP kernels for gfx950 (CDNA4, wave64) of the Wedge-Frontier pull engine.
//
// Steps of one iteration (Wedge Overview, Fig. 5 control loop):
//   k_translate      frontier -> Wedge Frontier bitmap (Frontier Transformation)
//   k_bitmap_compact Wedge bitmap -> marked-chunk list; frontier bitmap ->
//                    next frontier list + out-degree prefix (+ commit)
//   k_pull_*         destination-oriented gather/reduce over the marked chunks
//                    or over every in-edge (Background, Push vs. Pull)
// and the PageRank full pull with its epilogue.
//
// Every kernel is memory-bound: nothing here is a dense contraction.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace wedge {
namespace {

using namespace dev;


// ------------------------------------------------------------ small kernels

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t count, uint32_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_clear(ClearList l) {
    const int r = blockIdx.y;
    uint32_t* p = l.p[r];
    const uint64_t n = l.words[r];
    const uint64_t n4 = n / 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint4* p4 = reinterpret_cast<uint4*>(p);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        p4[i] = make_uint4(0u, 0u, 0u, 0u);
    for (uint64_t i = n4 * 4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// One wave: lanes 0..15 copy the 64-byte counter block to host memory, then
// (clear) lanes 0..5 zero fnext, marked and ftotal. The system-scope fence
// waits until the wave's stores are visible to the host; only then does lane
// 0 store the sequence number the host polls for.
__global__ void k_publish_ctl(Ctl* __restrict__ ctl, Ctl* __restrict__ host, int clear,
                              uint64_t* __restrict__ seq_host, uint64_t seq) {
    static_assert(sizeof(Ctl) == 64, "64-byte counter block");
    const uint32_t lane = threadIdx.x;
    uint32_t* c = reinterpret_cast<uint32_t*>(ctl);
    uint32_t* h = reinterpret_cast<uint32_t*>(host);
    if (lane < 16) {
        const uint32_t v = c[lane];
        if (h) h[lane] = v;
        if (clear && lane < 6) c[lane] = 0u;
    }
    __threadfence_system();
    if (seq_host && lane == 0) {
        *reinterpret_cast<volatile uint64_t*>(seq_host) = seq;
        __threadfence_system();
    }
}

__global__ void k_iota_u32(uint32_t* __restrict__ p, uint32_t count) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = i;
}

// F_0 = {src}: value 0 at the source in one or two value arrays, and the
// source's bit in the current-frontier bitmap.
__global__ void k_seed_source(uint32_t src, const uint32_t* __restrict__ row_off,
                              uint32_t* val_a, uint32_t* val_b, uint32_t* flist, uint32_t* degpre,
                              uint64_t* fcur, uint32_t* csum, Ctl* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        val_a[src] = 0;
        if (val_b) val_b[src] = 0;
        flist[0] = src;
        degpre[0] = 0;
        set_bit_sum(fcur, csum, src);
        const unsigned long long d = row_off[src + 1] - row_off[src];
        ctl->fnext = ((d ? 1ull : 0ull) << kDegBits) | d;
        ctl->ftotal = 1;
        ctl->marked = 0;
    }
}

// F_0 = V with label(v) = the vertex's caller id (inv maps internal ids back;
// null = identity); the out-degree prefix of the identity list is row_off.
__global__ void k_seed_all(uint32_t n, uint32_t m, const uint32_t* __restrict__ row_off,
                           const uint32_t* __restrict__ inv, uint32_t* __restrict__ label,
                           uint32_t* __restrict__ val_prev, uint32_t* __restrict__ flist,
                           uint32_t* __restrict__ degpre, uint64_t* __restrict__ fcur,
                           uint32_t* __restrict__ csum, Ctl* ctl) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t id = inv ? inv[v] : v;
        label[v] = id;
        val_prev[v] = id;
        flist[v] = v;
        degpre[v] = row_off[v];
    }
    const uint32_t words = (n + 63) / 64;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) {
        const uint32_t left = n - i * 64;
        fcur[i] = left >= 64 ? ~0ull : ((1ull << left) - 1ull);
        if (csum && (i & 63) == 0) csum[i >> 6] = 1u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->fnext = ((unsigned long long)n << kDegBits) | (unsigned long long)m;
        ctl->ftotal = n;
        ctl->marked = 0;
    }
}

// out[v] = val[perm[v]]: internal order back to the caller's ids (coalesced
// writes, gathered reads).
template <typename T>
__global__ void k_unpermute(uint32_t n, const uint32_t* __restrict__ perm,
                            const T* __restrict__ val, T* __restrict__ out) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        out[v] = val[perm[v]];
}

// ------------------------------------------------- frontier transformation
//
// For every out-edge of every frontier vertex (Frontier Transformation: look
// the vertex up in the edge index and set the bits it lists), set the Wedge
// Frontier bit of the chunk holding that edge's in-edge position. Work is
// balanced by edges, not vertices: lane j of wave w takes edge
// a = w*64*EPT + i*64 + j of the concatenated out-edge lists (degpre is the
// exclusive out-degree prefix over the list), so a high-degree vertex is split
// across many waves. Lanes that hit the same bitmap word are merged in the
// wave, and one atomicOr per distinct word is issued.
template <int EPT>
__global__ __launch_bounds__(kBlock) void k_translate(const uint32_t* __restrict__ flist,
                                                      const uint32_t* __restrict__ degpre,
                                                      uint32_t fcount, uint32_t active,
                                                      const uint32_t* __restrict__ row_off,
                                                      const uint32_t* __restrict__ pos, int lc,
                                                      uint32_t* __restrict__ wbits32,
                                                      uint32_t* __restrict__ wsum) {
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    translate_wave<EPT>(wave, flist, degpre, fcount, active, row_off, pos, lc, wbits32, wsum);
}

// ------------------------------------------------------- bitmap compaction
//
// Turns a bitmap into a list of its set bit indices. Each wave owns G
// consecutive 64-bit words; lane l stands for bit l of a word, so a popcount
// of the word below the lane gives each set bit its rank. One atomicAdd per
// block reserves the output range. Words are cleared after reading so the
// bitmap is all-zero for its next use; *total counts every set bit.
//   DEG:    list only vertices with out-edges (the only ones the translation
//           needs), with the exclusive out-degree prefix, and sum their
//           out-degrees (the next frontier's A).
//   COMMIT: also copy val[v] to val_prev[v] for every listed vertex.
//   COPY:   also copy every word to copy_to (the next-frontier bitmap becomes
//           the current one while it is cleared).
// Counter layout: (count << 33) | out-degree sum.
template <bool DEG, bool COMMIT, bool COPY, int G>
__global__ __launch_bounds__(kCompactWaves * 64) void k_bitmap_compact(
    uint64_t* __restrict__ bits, uint64_t words, uint32_t limit,
    const uint32_t* __restrict__ row_off, uint32_t* __restrict__ list,
    uint32_t* __restrict__ degpre, unsigned long long* counter, unsigned long long* total,
    uint32_t* __restrict__ val_prev, const uint32_t* __restrict__ val,
    uint64_t* __restrict__ copy_to, uint32_t* __restrict__ sum_bits, uint32_t* __restrict__ sum_copy) {
    bitmap_compact_block<DEG, COMMIT, COPY, G, kCompactWaves>(blockIdx.x, bits, words, limit, row_off,
                                                              list, degpre, counter, total, val_prev,
                                                              val, copy_to, sum_bits, sum_copy);
}

// The finalisation after a full pull, which sets no bits: the next frontier
// is every vertex with val < val_prev (COMMIT: CC and SSSP, the vertices the
// pull lowered) or with val == level (BFS, the vertices the pull reached),
// listed (and committed) as k_bitmap_compact does for the bits a pull sets.
template <bool COMMIT, int G>
__global__ __launch_bounds__(kCompactWaves * 64) void k_finalize_from_values(
    uint64_t* __restrict__ bits, uint64_t words, uint32_t limit,
    const uint32_t* __restrict__ row_off, uint32_t* __restrict__ list,
    uint32_t* __restrict__ degpre, unsigned long long* counter, unsigned long long* total,
    uint32_t* __restrict__ val_prev, const uint32_t* __restrict__ val,
    uint64_t* __restrict__ copy_to, uint32_t* __restrict__ sum_bits, uint32_t* __restrict__ sum_copy,
    uint32_t level) {
    bitmap_compact_block<true, COMMIT, true, G, kCompactWaves, true>(blockIdx.x, bits, words, limit, row_off,
                                                                    list, degpre, counter, total, val_prev,
                                                                    val, copy_to, sum_bits, sum_copy, level);
}

// ------------------------------------------------------------- the pulls
//
// One lane per in-edge position. A lane reads its destination from the row
// layout and its source from the streamed in-edge array, and forms the
// candidate value the edge carries. Lanes of one destination are reduced in
// the wave (min), and the segment head applies the result:
//   BFS  : destinations already visited are skipped before their in-edges are
//          read (Evaluation, no-frontier BFS iterations get cheaper); an
//          unvisited destination with an in-neighbour in the current frontier
//          (a bit test in the 1-bit-per-vertex frontier, the check a pull
//          engine makes after reading an edge; Background, Push vs. Pull) gets
//          k+1.
//   CC   : candidate = label_prev[u].
//   SSSP : candidate = dist_prev[u] + w (u reached).
// CC and SSSP gather the source value without a frontier test: the value is
// one random read either way, and an edge from outside the frontier cannot
// lower its destination (below).
// An improvement lowers val[v] with atomicMin (a destination can span several
// chunks and waves) and sets v's bit in the next-frontier bitmap. Values are
// read from val_prev, the copy committed at the end of the previous
// iteration, so every iteration sees one consistent snapshot; BFS only ever
// writes k+1 and only reads "== k", so it can use a single array.
// Superfluous edges (chunk members that are not active) never lower a value,
// which is why any chunk granularity, or none, gives the same result
// (Frontier Transformation, "Frontier Precision").
// Full pull: wave w covers rows [w*R, w*R + R), i.e. every in-edge once.
template <int APP, int R, bool INPLACE = false>
__global__ __launch_bounds__(kBlock) WEDGE_PULL_OCCUPANCY void k_pull_full(GraphArgs g, uint32_t iter,
                                                      uint32_t* __restrict__ val,
                                                      const uint32_t* __restrict__ val_prev,
                                                      const uint64_t* __restrict__ fcur,
                                                      uint64_t* __restrict__ fbits,
                                                      uint32_t* __restrict__ fsum) {
    const int lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t r0 = wave * R;
    if (r0 >= g.rows) return;
    uint32_t p[R];
    bool valid[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint64_t pp = (r0 + i) * 64 + lane;
        valid[i] = pp < g.m;
        p[i] = (uint32_t)pp;
    }
    static_assert(APP != kBfs, "the BFS full pull is k_pull_full_bfs");
    pull_lanes<APP, R, true, INPLACE, CanonicalEdges, false>(g, p, valid, iter, val, val_prev, fcur, fbits, fsum);
}

// BFS full pull: each block first copies the first `words` 32-bit words of
// the current frontier bitmap into LDS (with out-degree-sorted ids, the bits
// of the sources of most in-edges: on R-MAT scale 24 the first 2^19 ids
// source about two thirds of them); the frontier tests of those sources are
// served by LDS. Waves then stride over R-row tiles.
template <int R>
__global__ __launch_bounds__(kHotBlock) void k_pull_full_bfs(GraphArgs g, uint32_t iter,
                                                             uint32_t* __restrict__ val,
                                                             const uint64_t* __restrict__ fcur,
                                                             uint64_t* __restrict__ fbits,
                                                             uint32_t* __restrict__ fsum, uint32_t words) {
    extern __shared__ uint32_t s_bits[];
    {
        const uint32_t* f32 = reinterpret_cast<const uint32_t*>(fcur);
        constexpr int kPer = (int)((kHotVerts + kHotBlock - 1) / kHotBlock);
        uint32_t t[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * kHotBlock;
            t[k] = f32[i < words ? i : 0u];
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * kHotBlock;
            if (i < words) s_bits[i] = t[k];
        }
    }
    __syncthreads();
    HotFrontierEdges edges;
    edges.words = words;
    edges.s_bits = s_bits;
    const int lane = lane_id();
    const uint64_t wpb = kHotBlock / 64;
    const uint64_t stride = (uint64_t)gridDim.x * wpb;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint64_t w = blockIdx.x * wpb + wib;; w += stride) {
        const uint64_t r0 = w * R;
        if (r0 >= g.rows) break;
        uint32_t p[R];
        bool valid[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint64_t pp = (r0 + i) * 64 + lane;
            valid[i] = pp < g.m;
            p[i] = (uint32_t)pp;
        }
        pull_lanes<kBfs, R, true, false, HotFrontierEdges, false>(g, p, valid, iter, val, nullptr, fcur,
                                                                  fbits, fsum, edges);
    }
}

// Full pull over one slice of the source-sliced copy (CC and SSSP). The pull
// over every in-edge is run slice after slice, one launch each, over the whole
// GPU: during a launch every XCD gathers only the values of that slice's
// sources (an eighth of the value array), so they stay in its L2. In the
// synchronous pull each block first copies the committed values of the
// slice's first `hot` sources (slice-local ids, its highest out-degrees) into
// LDS, where their gathers are served; the in-place pull reads the values as
// they fall and stages nothing. Waves then stride over R-row tiles, each
// pulled exactly like the canonical array (wave-owned destinations take a
// plain store, the tile's first and last segments a min-atomic); successive
// launches lower the same destinations in turn. PACKED: each position holds
// (slice-local source << 8) | weight.
template <int APP, int R, bool INPLACE, bool PACKED>
__global__ __launch_bounds__(kHotBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_pull_slice(
    GraphArgs g, uint32_t slice, uint32_t lg, uint32_t row_begin, uint32_t row_end, uint32_t edge_end, uint32_t iter,
    uint32_t* __restrict__ val, const uint32_t* __restrict__ val_prev,
    const uint64_t* __restrict__ fcur, uint64_t* __restrict__ fbits, uint32_t* __restrict__ fsum,
    uint32_t hot) {
    extern __shared__ uint32_t s_val[];
    if (!INPLACE) {
        // all of a thread's loads are issued before its first store
        constexpr int kPer = (int)((kHotVerts + kHotBlock - 1) / kHotBlock);
        uint32_t t[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * kHotBlock;
            const uint32_t gi = xcd_slice_global(i < hot ? i : 0u, slice, lg);
            t[k] = val_prev[gi < g.n ? gi : 0u];
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * kHotBlock;
            if (i < hot) s_val[i] = t[k];
        }
        __syncthreads();
    }
    const SliceEdges<PACKED, !INPLACE> edges{slice, lg, g.n, INPLACE ? 0u : hot, s_val};
    const int lane = lane_id();
    const uint64_t wpb = kHotBlock / 64;
    const uint64_t stride = (uint64_t)gridDim.x * wpb;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint64_t w = blockIdx.x * wpb + wib;; w += stride) {
        const uint64_t r0 = (uint64_t)row_begin + w * R;
        if (r0 >= row_end) break;
        uint32_t p[R];
        bool valid[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint64_t pp = (r0 + i) * 64 + lane;
            valid[i] = pp < edge_end;
            p[i] = (uint32_t)pp;
        }
        pull_lanes<APP, R, true, INPLACE, SliceEdges<PACKED, !INPLACE>, false>(g, p, valid, iter, val, val_prev,
                                                                             fcur, fbits, fsum, edges);
    }
}

// Pull over the marked chunks: the chunk list holds K = *marked chunk ids of
// 2^lc positions each. A 64-lane slot covers 64 >> lc chunks (lc <= 6) or one
// 64-position part of a chunk (lc > 6). Waves stride over the slots, R slots at
// a time; K is read on the device, so the launch needs no host round trip.
template <int APP, int R, int FORM, bool INPLACE = false>
__global__ __launch_bounds__(kBlock) WEDGE_CHUNK_OCCUPANCY void k_pull_chunks(GraphArgs g, uint32_t iter, int lc,
                                                        const uint32_t* __restrict__ list,
                                                        const unsigned long long* marked,
                                                        uint32_t* __restrict__ val,
                                                        const uint32_t* __restrict__ val_prev,
                                                        const uint64_t* __restrict__ fcur,
                                                        uint64_t* __restrict__ fbits,
                                                        uint32_t* __restrict__ fsum) {
    const int lane = lane_id();
    const uint64_t K = *marked >> kDegBits;
    const uint64_t slots = chunk_slots(K, lc);
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t s0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * R; s0 < slots;
         s0 += nwaves * R) {
        uint32_t p[R];
        bool valid[R];
        chunk_slot_rows<R, FORM>(s0, slots, lane, lc, list, K, g.m, p, valid);
        pull_lanes<APP, R, false, INPLACE>(g, p, valid, iter, val, val_prev, fcur, fbits, fsum);
    }
}

// ---------------------------------------------------------------- PageRank
//
// Full pull of PageRank (no frontier): S(v) = sum over in-edges of
// contrib(u) = r(u)/outdeg(u). A wave owns a tile of kPrTileRows rows; sums
// are formed by segmented tree reductions per row, carried across the rows of
// the tile in order, and written straight to S for destinations that lie
// inside the tile. A destination crossing a tile boundary leaves its partial
// from the tile where it starts in tail[tile] and its partials from later tiles
// in head[tile]; k_pr_fixup adds them in a fixed order. No float atomics: the
// result is deterministic.
// ACCUM: interior destinations are added to sum instead of written (the
// sliced pull adds each slice's partial sums in turn).
template <int R, int B, bool ACCUM = false, class Gather>
__device__ __forceinline__ void pr_tile(const GraphArgs& g, uint64_t tile, Gather gather,
                                        float* __restrict__ sum, float* __restrict__ head_part,
                                        float* __restrict__ tail_part) {
    static_assert(R % B == 0, "rows are loaded in batches of B");
    const int lane = lane_id();
    const uint64_t r0 = tile * R;  // wave-uniform
    if (r0 >= g.rows) return;
    float carry = 0.0f;
    bool from_before = false;
    // Rows are loaded B at a time and reduced in order; the carry links
    // segments across rows and batches. Loads are branch-free (a lane past
    // the last edge reads the last position and is masked) so that the
    // batch's memory round trips overlap. Which lanes hold an edge, and where
    // segments start, are wave-uniform masks built by the scalar unit from
    // the row's mask and the edge count.
#pragma unroll
    for (int i0 = 0; i0 < R; i0 += B) {
        if (r0 + i0 >= g.rows) break;
        uint32_t pc[B], u[B], dst[B], sg[B];
        uint64_t mk[B + 1];
        float x[B];
        // the rows' layout: scalar loads (rows past the end read the layout's
        // padding, whose mask 1 marks a segment start)
        row_layout<B>(g, r0 + i0, mk, sg);
#pragma unroll
        for (int j = 0; j < B; ++j) pc[j] = (uint32_t)umin64((r0 + i0 + j) * 64 + lane, g.m - 1);
#pragma unroll
        for (int j = 0; j < B; ++j) u[j] = ld_stream(g.in_src + pc[j]);
        // a lane's segment is counted with mbcnt over the row's mask
#pragma unroll
        for (int j = 0; j < B; ++j) dst[j] = dst_of_whole_row(g, mk[j], sg[j]);
        // dst is only used by the head lanes' stores; pinning it here keeps
        // the compiler from sinking its loads into those branches, which
        // would serialise them row by row
#pragma unroll
        for (int j = 0; j < B; ++j) __asm__ volatile("" : "+v"(dst[j]));
#pragma unroll
        for (int j = 0; j < B; ++j) x[j] = gather(u[j]);
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int i = i0 + j;
            const uint64_t r = r0 + i;
            if (r >= g.rows) break;
            // edges from this row's first position on (none in the rows that
            // pad a slice up to its aligned end); lanes past the last edge hold
            // none, and the first of them starts a segment of its own
            const uint64_t left = g.m > r * 64 ? g.m - r * 64 : 0ull;
            const uint64_t vmask = left >= 64 ? ~0ull : ((1ull << left) - 1ull);
            const uint64_t heads = mk[j] | 1ull | (left >= 64 ? 0ull : (1ull << left));
            const bool cont_in = !(mk[j] & 1ull);
            const bool cont_out = left > 64 && !(mk[j + 1] & 1ull);
            const bool last_row = (i == R - 1) || (r + 1 >= g.rows);
            float s = seg_reduce(lane_bit(vmask) ? x[j] : 0.0f, heads,
                                 [](float a, float b) { return a + b; });
            if (i == 0) from_before = cont_in;
            if (lane == 0 && cont_in) s = carry + s;
            const uint64_t hv = heads & vmask;
            const int h_last = 63 - __clzll(hv);
            if (lane_bit(hv)) {
                const bool seg_before = lane == 0 && cont_in && from_before;
                if (lane == h_last && cont_out) {
                    if (last_row) {
                        if (seg_before) head_part[tile] = s;
                        else tail_part[tile] = s;
                    }
                } else if (seg_before) {
                    head_part[tile] = s;
                } else {
                    if (ACCUM) sum[dst[j]] += s;
                    else sum[dst[j]] = s;
                }
            }
            const float last_s = lane_bcast(s, h_last);
            const bool nfb = h_last == 0 && cont_in && from_before;
            if (cont_out && !last_row) {
                carry = last_s;
                from_before = nfb;
            }
        }
    }
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_pr_pull(GraphArgs g, const float* __restrict__ contrib,
                                                    float* __restrict__ sum,
                                                    float* __restrict__ head_part,
                                                    float* __restrict__ tail_part) {
    const uint64_t tile = (uint64_t)blockIdx.x * kWavesPerBlock +
                          __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    pr_tile<R, R>(g, tile, [&](uint32_t u) { return contrib[u]; }, sum, head_part, tail_part);
}

// The same pull with the first `hot` contributions held in LDS. Vertices are
// numbered by descending out-degree, so the lowest ids are the sources of the
// most in-edges (on R-MAT scale 24 the first 16384 source about 29% of them);
// their gathers are served by LDS, and the global gather of such a lane is
// pointed at one shared address. Each block copies contrib[0, hot) once and
// then strides over the tiles; tile results are the same as k_pr_pull's.
template <int R>
__global__ __launch_bounds__(kHotBlock) void k_pr_pull_hot(GraphArgs g, const float* __restrict__ contrib,
                                                           float* __restrict__ sum,
                                                           float* __restrict__ head_part,
                                                           float* __restrict__ tail_part,
                                                           uint32_t hot, uint64_t tiles) {
    extern __shared__ float s_hot[];  // hot values + one spare 16-byte slot
    {
        // all of a thread's 16-byte loads are issued before its first store;
        // the stores are unconditional, a thread past the end writing the
        // spare slot
        constexpr int kPer = (int)((kHotVerts / 4 + kHotBlock - 1) / kHotBlock);
        const uint32_t hot4 = hot / 4;
        const float4* src4 = reinterpret_cast<const float4*>(contrib);
        float4* dst4 = reinterpret_cast<float4*>(s_hot);
        const uint32_t spare = (hot + 3) / 4;
        float4 t[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * kHotBlock;
            t[k] = src4[i < hot4 ? i : 0u];
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * kHotBlock;
            dst4[i < hot4 ? i : spare] = t[k];
        }
        for (uint32_t i = hot4 * 4 + threadIdx.x; i < hot; i += kHotBlock) s_hot[i] = contrib[i];
    }
    __syncthreads();
    const uint64_t wpb = kHotBlock / 64;
    const uint64_t stride = (uint64_t)gridDim.x * wpb;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint64_t t = blockIdx.x * wpb + wib; t < tiles; t += stride)
        pr_tile<R, kHotBatch>(
            g, t,
            [&](uint32_t u) {
                const float gv = contrib[u < hot ? 0u : u];
                const float lv = s_hot[u < hot ? u : 0u];
                return u < hot ? lv : gv;
            },
            sum, head_part, tail_part);
}


// PageRank pull over one slice of the source-sliced copy: the slices are
// pulled one launch after another and each adds its partial sums into S, in
// slice order (deterministic). Each block first copies the contributions of
// the slice's first `hot` sources (its highest out-degree ones) into LDS; a
// launch gathers only this slice's sources, so the rest of its gathers stay in
// the L2. Segments crossing a tile boundary leave their parts in head/tail;
// k_pr_fixup_xs adds them afterwards.
template <int R, bool PACKED>
__global__ __launch_bounds__(kHotBlock) void k_pr_pull_slice(GraphArgs g, uint32_t lg,
                                                             uint64_t tile_begin, uint64_t tile_end,
                                                             const float* __restrict__ cs,
                                                             float* __restrict__ sum,
                                                             float* __restrict__ head_part,
                                                             float* __restrict__ tail_part,
                                                             uint32_t hot) {
    // cs: this slice's contributions, indexed by slice-local id (every id an
    // in-edge word can hold is below the capacity cs spans)
    extern __shared__ float s_hot[];
    {
        constexpr int kPer = (int)((kHotVerts + kHotBlock - 1) / kHotBlock);
        float t[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * kHotBlock;
            t[k] = cs[i < hot ? i : 0u];
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = threadIdx.x + (uint32_t)k * kHotBlock;
            if (i < hot) s_hot[i] = t[k];
        }
    }
    __syncthreads();
    const uint64_t wpb = kHotBlock / 64;
    const uint64_t stride = (uint64_t)gridDim.x * wpb;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint64_t t = tile_begin + blockIdx.x * wpb + wib; t < tile_end; t += stride)
        pr_tile<R, kHotBatch, true>(
            g, t,
            [&](uint32_t word) {
                const uint32_t l = PACKED ? (word >> 8) : xcd_slice_local(word, lg);
                const bool h = l < hot;
                const float gv = cs[h ? 0u : l];
                const float lv = s_hot[h ? l : 0u];
                return h ? lv : gv;
            },
            sum, head_part, tail_part);
}

// Crossing segments of the sliced pull: one lane per destination with few
// crossing tiles, one wave per destination with many; each adds, in slice
// order and tile order, the tail part of every crossing segment and the head
// parts of the tiles it runs into, then adds the total to S. The last block
// of the long launch reduces the previous epilogue's dangling partials.
__global__ __launch_bounds__(kBlock) void k_pr_fixup_xs_short(const uint32_t* __restrict__ vs,
                                                              const uint32_t* __restrict__ off,
                                                              const uint32_t* __restrict__ tt,
                                                              uint64_t count,
                                                              const float* __restrict__ head_part,
                                                              const float* __restrict__ tail_part,
                                                              float* __restrict__ sum) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float acc = 0.0f;
    for (uint32_t q = off[e]; q < off[e + 1]; ++q) {
        const uint32_t ta = tt[2 * q], tb = tt[2 * q + 1];
        acc += tail_part[ta];
        for (uint32_t t = ta + 1; t <= tb; ++t) acc += head_part[t];
    }
    sum[vs[e]] += acc;
}

__global__ __launch_bounds__(kBlock) void k_pr_fixup_xs_long(const uint32_t* __restrict__ vs,
                                                             const uint32_t* __restrict__ off,
                                                             const uint32_t* __restrict__ tt,
                                                             uint64_t first, uint64_t count,
                                                             const float* __restrict__ head_part,
                                                             const float* __restrict__ tail_part,
                                                             float* __restrict__ sum,
                                                             const double* __restrict__ partials,
                                                             uint32_t parts, double* __restrict__ dnext) {
    const int lane = lane_id();
    if (blockIdx.x == gridDim.x - 1) {
        __shared__ double s_part[kWavesPerBlock];
        if (!dnext) return;
        double acc = 0.0;
        for (uint32_t i = threadIdx.x; i < parts; i += blockDim.x) acc += partials[i];
        acc = wave_sum_tree(acc);
        if (lane == 0) s_part[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < kWavesPerBlock; ++i) t += s_part[i];
            *dnext = t;
        }
        return;
    }
    const uint64_t e = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (e >= count) return;
    const uint64_t k = first + e;
    float acc = 0.0f;
    for (uint32_t q = off[k]; q < off[k + 1]; ++q) {
        const uint32_t ta = tt[2 * q], tb = tt[2 * q + 1];
        if (lane == 0) acc += tail_part[ta];
        for (uint32_t t = ta + 1 + lane; t <= tb; t += 64) acc += head_part[t];
    }
    acc = wave_sum_tree(acc);
    if (lane == 0) sum[vs[k]] += acc;
}

// S(v) = tail[first tile] + sum of head[t] over the later tiles v covers.
// Short spans: one lane each, summed in tile order.
__global__ __launch_bounds__(kBlock) void k_pr_fixup_short(const uint32_t* __restrict__ spans,
                                                           uint64_t nspans,
                                                           const float* __restrict__ head_part,
                                                           const float* __restrict__ tail_part,
                                                           float* __restrict__ sum) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nspans) return;
    const uint32_t v = spans[3 * e], ta = spans[3 * e + 1], tb = spans[3 * e + 2];
    float acc = tail_part[ta];
    for (uint32_t t = ta + 1; t <= tb; ++t) acc += head_part[t];
    sum[v] = acc;
}

// Long spans: one wave each, lane-strided partial sums then a fixed tree.
// The grid's last block instead reduces the dangling-mass partials of the
// previous epilogue into *dnext, in a fixed order.
__global__ __launch_bounds__(kBlock) void k_pr_fixup_long(const uint32_t* __restrict__ spans,
                                                          uint64_t nspans,
                                                          const float* __restrict__ head_part,
                                                          const float* __restrict__ tail_part,
                                                          float* __restrict__ sum,
                                                          const double* __restrict__ partials,
                                                          uint32_t parts, double* __restrict__ dnext) {
    const int lane = lane_id();
    if (blockIdx.x == gridDim.x - 1) {
        __shared__ double s_part[kWavesPerBlock];
        if (!dnext) return;
        double acc = 0.0;
        for (uint32_t i = threadIdx.x; i < parts; i += blockDim.x) acc += partials[i];
        acc = wave_sum_tree(acc);
        if (lane == 0) s_part[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < kWavesPerBlock; ++i) t += s_part[i];
            *dnext = t;
        }
        return;
    }
    const uint64_t e = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (e >= nspans) return;
    const uint32_t v = spans[3 * e], ta = spans[3 * e + 1], tb = spans[3 * e + 2];
    float acc = 0.0f;
    for (uint32_t t = ta + 1 + lane; t <= tb; t += 64) acc += head_part[t];
    acc = wave_sum_tree(acc);
    if (lane == 0) sum[v] = tail_part[ta] + acc;
}

// Position of vertex v's contribution: vertex order (cap = 0) or slice-major
// (see xs_contrib_cap).
__device__ __forceinline__ uint64_t contrib_pos(uint32_t v, uint32_t lg, uint64_t cap) {
    return cap ? (uint64_t)xcd_slice_of(v, lg) * cap + xcd_slice_local(v, lg) : (uint64_t)v;
}

__global__ void k_pr_init(uint32_t n, const uint32_t* __restrict__ row_off, float* __restrict__ rank,
                          float* __restrict__ contrib, float* __restrict__ sum, uint32_t lg, uint64_t cap) {
    const float r0 = 1.0f / (float)n;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t od = row_off[v + 1] - row_off[v];
        rank[v] = r0;
        contrib[contrib_pos(v, lg, cap)] = od ? r0 / (float)od : 0.0f;
        sum[v] = 0.0f;
    }
}

__global__ void k_set_f64(double* p, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// r'(v) = (1-d)/n + d (S(v) + D/n); contrib'(v) = r'/outdeg; per-block sum of
// the new rank mass on out-degree-0 vertices (the next D), in FP64. Each block
// covers a fixed contiguous vertex range, so the partials (and their order)
// do not depend on timing. S is cleared once read, so that a pull that adds
// into it (the sliced pull) starts from zero.
__global__ __launch_bounds__(kBlock) void k_pr_epilogue(uint32_t n, uint32_t per_block,
                                                        const uint32_t* __restrict__ row_off,
                                                        float* __restrict__ sum, double d,
                                                        const double* __restrict__ dcur,
                                                        float* __restrict__ rank,
                                                        float* __restrict__ contrib,
                                                        double* __restrict__ partials, uint32_t lg,
                                                        uint64_t cap) {
    __shared__ double s_part[kWavesPerBlock];
    const double dn = *dcur / (double)n;
    const double base = (1.0 - d) / (double)n;
    const uint32_t lo = blockIdx.x * per_block;
    const uint32_t hi = min(n, lo + per_block);
    double acc = 0.0;
    for (uint32_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
        const float r = (float)(base + d * ((double)sum[v] + dn));
        sum[v] = 0.0f;
        const uint32_t od = row_off[v + 1] - row_off[v];
        rank[v] = r;
        contrib[contrib_pos(v, lg, cap)] = od ? r / (float)od : 0.0f;
        if (!od) acc += (double)r;
    }
    acc = wave_sum_tree(acc);
    if (lane_id() == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kWavesPerBlock; ++i) t += s_part[i];
        partials[blockIdx.x] = t;
    }
}

uint32_t grid_for(uint64_t threads, uint32_t cap = 1u << 20) {
    uint64_t b = (threads + kBlock - 1) / kBlock;
    if (b == 0) b = 1;
    return (uint32_t)(b < cap ? b : cap);
}

}  // namespace

// ------------------------------------------------------------- launchers

hipError_t launch_clear(const ClearList& l, hipStream_t s) {
    if (!l.count) return hipSuccess;
    uint64_t most = 0;
    for (int i = 0; i < l.count; ++i) {
        if (reinterpret_cast<uintptr_t>(l.p[i]) & 15u) return hipErrorInvalidValue;
        most = std::max(most, l.words[i]);
    }
    const uint64_t blocks = std::min<uint64_t>(2048, std::max<uint64_t>(1, (most / 4 + kBlock - 1) / kBlock));
    k_clear<<<dim3((uint32_t)blocks, (uint32_t)l.count), kBlock, 0, s>>>(l);
    return hipGetLastError();
}

hipError_t launch_publish_ctl(Ctl* ctl, Ctl* host_dev, bool clear, uint64_t* seq_dev, uint64_t seq,
                              hipStream_t s) {
    if (!ctl) return hipErrorInvalidValue;
    k_publish_ctl<<<1, 64, 0, s>>>(ctl, host_dev, clear ? 1 : 0, seq_dev, seq);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s) {
    if (!count) return hipSuccess;
    k_fill_u32<<<grid_for(count, 8192), kBlock, 0, s>>>(p, count, value);
    return hipGetLastError();
}

hipError_t launch_iota_u32(uint32_t* p, uint32_t count, hipStream_t s) {
    if (!count) return hipSuccess;
    k_iota_u32<<<grid_for(count, 8192), kBlock, 0, s>>>(p, count);
    return hipGetLastError();
}

hipError_t launch_seed_source(uint32_t src, const uint32_t* row_off, uint32_t* val_a,
                              uint32_t* val_b, uint32_t* flist, uint32_t* degpre, uint64_t* fcur,
                              uint32_t* csum, Ctl* ctl, hipStream_t s) {
    k_seed_source<<<1, 64, 0, s>>>(src, row_off, val_a, val_b, flist, degpre, fcur, csum, ctl);
    return hipGetLastError();
}

hipError_t launch_seed_all(uint32_t n, uint64_t m, const uint32_t* row_off, const uint32_t* inv,
                           uint32_t* label, uint32_t* val_prev, uint32_t* flist, uint32_t* degpre,
                           uint64_t* fcur, uint32_t* csum, Ctl* ctl, hipStream_t s) {
    k_seed_all<<<grid_for(n, 8192), kBlock, 0, s>>>(n, (uint32_t)m, row_off, inv, label, val_prev,
                                                    flist, degpre, fcur, csum, ctl);
    return hipGetLastError();
}

hipError_t launch_unpermute_u32(uint32_t n, const uint32_t* perm, const uint32_t* val,
                                uint32_t* out, hipStream_t s) {
    if (!n) return hipSuccess;
    k_unpermute<uint32_t><<<grid_for(n, 16384), kBlock, 0, s>>>(n, perm, val, out);
    return hipGetLastError();
}

hipError_t launch_unpermute_f32(uint32_t n, const uint32_t* perm, const float* val, float* out,
                                hipStream_t s) {
    if (!n) return hipSuccess;
    k_unpermute<float><<<grid_for(n, 16384), kBlock, 0, s>>>(n, perm, val, out);
    return hipGetLastError();
}

hipError_t launch_translate(const uint32_t* flist, const uint32_t* degpre, uint32_t fcount,
                            uint64_t active, const uint32_t* row_off, const uint32_t* pos,
                            int log_chunk, uint64_t* wbits, uint32_t* wsum, hipStream_t s) {
    if (!fcount || !active) return hipSuccess;
    const uint64_t waves = (active + 64ull * kTranslateEpt - 1) / (64ull * kTranslateEpt);
    const uint64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    k_translate<kTranslateEpt><<<(uint32_t)blocks, kBlock, 0, s>>>(
        flist, degpre, fcount, (uint32_t)active, row_off, pos, log_chunk,
        reinterpret_cast<uint32_t*>(wbits), wsum);
    return hipGetLastError();
}

hipError_t launch_compact_chunks(uint64_t* wbits, uint64_t words, uint32_t* list, Ctl* ctl,
                                 uint32_t* wsum, hipStream_t s) {
    if (!words) return hipSuccess;
    const uint64_t waves = (words + kCompactWords - 1) / kCompactWords;
    const uint32_t blocks = (uint32_t)((waves + kCompactWaves - 1) / kCompactWaves);
    k_bitmap_compact<false, false, false, kCompactWords><<<blocks, kCompactWaves * 64, 0, s>>>(
        wbits, words, 0xFFFFFFFFu, nullptr, list, nullptr, &ctl->marked, nullptr, nullptr, nullptr,
        nullptr, wsum, nullptr);
    return hipGetLastError();
}

hipError_t launch_finalize(uint64_t* fbits, uint32_t n, const uint32_t* row_off, uint32_t* flist,
                           uint32_t* degpre, Ctl* ctl, uint32_t* val_prev, const uint32_t* val,
                           uint64_t* fcur, uint32_t* fsum, uint32_t* csum, hipStream_t s,
                           bool from_values, uint32_t level) {
    const uint64_t words = ((uint64_t)n + 63) / 64;
    if (!words) return hipSuccess;
    const uint64_t waves = (words + kCompactWords - 1) / kCompactWords;
    const uint32_t blocks = (uint32_t)((waves + kCompactWaves - 1) / kCompactWaves);
    unsigned long long* c = &ctl->fnext;
    unsigned long long* t = &ctl->ftotal;
    if (from_values) {
        if (!val || !fcur) return hipErrorInvalidValue;
        if (val_prev)
            k_finalize_from_values<true, kCompactWords><<<blocks, kCompactWaves * 64, 0, s>>>(
                fbits, words, n, row_off, flist, degpre, c, t, val_prev, val, fcur, fsum, csum, 0u);
        else
            k_finalize_from_values<false, kCompactWords><<<blocks, kCompactWaves * 64, 0, s>>>(
                fbits, words, n, row_off, flist, degpre, c, t, nullptr, val, fcur, fsum, csum, level);
    } else if (val_prev && fcur)
        k_bitmap_compact<true, true, true, kCompactWords><<<blocks, kCompactWaves * 64, 0, s>>>(
            fbits, words, n, row_off, flist, degpre, c, t, val_prev, val, fcur, fsum, csum);
    else if (fcur)
        k_bitmap_compact<true, false, true, kCompactWords><<<blocks, kCompactWaves * 64, 0, s>>>(
            fbits, words, n, row_off, flist, degpre, c, t, nullptr, nullptr, fcur, fsum, csum);
    else
        k_bitmap_compact<true, false, false, kCompactWords><<<blocks, kCompactWaves * 64, 0, s>>>(
            fbits, words, n, row_off, flist, degpre, c, t, nullptr, nullptr, nullptr, fsum, nullptr);
    return hipGetLastError();
}

// Resident blocks per compute unit of a kernel at a block size and dynamic
// LDS size (the same on every MI355X); queried once per kernel (a
// function-local static, initialised safely across threads); 0 if the query
// fails.
template <auto KERNEL>
int resident_blocks(int block, size_t lds) {
    static const int b = [&] {
        int x = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&x, KERNEL, block, lds) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        return x;
    }();
    return b;
}

int slice_pull_resident(int app, bool inplace, bool packed, size_t lds) {
    if (app == kCc)
        return inplace ? resident_blocks<k_pull_slice<kCc, kPullRows, true, false>>(kHotBlock, lds)
                       : resident_blocks<k_pull_slice<kCc, kPullRows, false, false>>(kHotBlock, lds);
    if (packed)
        return inplace ? resident_blocks<k_pull_slice<kSssp, kPullRows, true, true>>(kHotBlock, lds)
                       : resident_blocks<k_pull_slice<kSssp, kPullRows, false, true>>(kHotBlock, lds);
    return inplace ? resident_blocks<k_pull_slice<kSssp, kPullRows, true, false>>(kHotBlock, lds)
                   : resident_blocks<k_pull_slice<kSssp, kPullRows, false, false>>(kHotBlock, lds);
}

// How many of slice j's first kHotVerts slice-local ids are vertices (the
// slice's groups in order; only the graph's last group can be partial).
uint32_t slice_hot_count(uint32_t n, uint32_t j, uint32_t lg) {
    constexpr uint32_t kGroup = 1u << kXcdGroupShift;
    uint32_t hot = 0;
    for (uint32_t i = 0; i < kHotVerts; i += kGroup) {
        const uint64_t first = xcd_slice_global(i, j, lg);
        if (first >= n) break;
        hot = i + (uint32_t)std::min<uint64_t>(kGroup, n - first);
    }
    return std::min(hot, kHotVerts);
}

// BFS pulls come in three shapes (rows per wave step); CC and SSSP in one.
template <int R>
uint32_t full_blocks(const DevGraph& g) {
    const uint64_t waves = (g.rows + R - 1) / R;
    return (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
}

hipError_t launch_pull_full(int app, const DevGraph& g, uint32_t iter, uint32_t* val,
                            const uint32_t* val_prev, const uint64_t* fcur, uint64_t* fbits,
                            uint32_t* fsum, hipStream_t s, int rows, bool inplace) {
    if (!g.rows) return hipSuccess;
    if (app != kBfs && rows != kPullRows) return hipErrorInvalidValue;
    if (inplace && app == kBfs) return hipErrorInvalidValue;
    if (app != kBfs && g.xs_rows) {
        const GraphArgs xa = xs_args_of(g);
        const size_t lds = inplace ? 0 : (size_t)kHotVerts * sizeof(uint32_t);
        const int per_cu = slice_pull_resident(app, inplace, g.xs_packed, lds);
        if (per_cu <= 0) return hipErrorInvalidConfiguration;
        for (int j = 0; j < (1 << g.xs_lg); ++j) {
            const uint32_t rb = g.xs_row_begin[j], re = g.xs_row_begin[j + 1];
            if (re == rb) continue;
            const uint64_t waves = ((uint64_t)(re - rb) + kPullRows - 1) / kPullRows;
            const uint32_t blocks = (uint32_t)std::min<uint64_t>(
                (uint64_t)std::max(g.cus, 1) * (uint64_t)per_cu, (waves + kHotBlock / 64 - 1) / (kHotBlock / 64));
            const uint32_t ee = g.xs_edge_end[j];
            const uint32_t hot = inplace ? 0u : slice_hot_count(g.n, (uint32_t)j, g.xs_lg);
#define WEDGE_SLICE_LAUNCH(A, IP, PK)                                                              \
    k_pull_slice<A, kPullRows, IP, PK><<<blocks, kHotBlock, lds, s>>>(xa, (uint32_t)j, g.xs_lg, rb, re, ee, iter, \
                                                                      val, val_prev, fcur, fbits, fsum, hot)
            if (app == kCc) {
                if (inplace) WEDGE_SLICE_LAUNCH(kCc, true, false);
                else WEDGE_SLICE_LAUNCH(kCc, false, false);
            } else if (g.xs_packed) {
                if (inplace) WEDGE_SLICE_LAUNCH(kSssp, true, true);
                else WEDGE_SLICE_LAUNCH(kSssp, false, true);
            } else {
                if (inplace) WEDGE_SLICE_LAUNCH(kSssp, true, false);
                else WEDGE_SLICE_LAUNCH(kSssp, false, false);
            }
#undef WEDGE_SLICE_LAUNCH
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    GraphArgs a = args_of(g);
    if (app == kBfs) {
        // resident blocks at the full LDS size, striding over the tiles
        const uint32_t words = (uint32_t)std::min<uint64_t>(kHotVerts, ((uint64_t)g.n + 31) / 32);
        const size_t lds = (size_t)kHotVerts * sizeof(uint32_t);
        int per_cu = 0;
        uint64_t tiles = 0;
        switch (rows) {
            case 4: per_cu = resident_blocks<k_pull_full_bfs<4>>(kHotBlock, lds); tiles = (g.rows + 3) / 4; break;
            case 16: per_cu = resident_blocks<k_pull_full_bfs<16>>(kHotBlock, lds); tiles = (g.rows + 15) / 16; break;
            case kPullRows:
                per_cu = resident_blocks<k_pull_full_bfs<kPullRows>>(kHotBlock, lds);
                tiles = (g.rows + kPullRows - 1) / kPullRows;
                break;
            default: return hipErrorInvalidValue;
        }
        if (per_cu <= 0) return hipErrorInvalidConfiguration;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((uint64_t)std::max(g.cus, 1) * (uint64_t)per_cu,
                                                             (tiles + kHotBlock / 64 - 1) / (kHotBlock / 64));
        switch (rows) {
            case 4: k_pull_full_bfs<4><<<blocks, kHotBlock, lds, s>>>(a, iter, val, fcur, fbits, fsum, words); break;
            case 16: k_pull_full_bfs<16><<<blocks, kHotBlock, lds, s>>>(a, iter, val, fcur, fbits, fsum, words); break;
            default: k_pull_full_bfs<kPullRows><<<blocks, kHotBlock, lds, s>>>(a, iter, val, fcur, fbits, fsum, words); break;
        }
    } else if (app == kCc) {
        if (inplace) k_pull_full<kCc, kPullRows, true><<<full_blocks<kPullRows>(g), kBlock, 0, s>>>(a, iter, val, val_prev, fcur, fbits, fsum);
        else k_pull_full<kCc, kPullRows><<<full_blocks<kPullRows>(g), kBlock, 0, s>>>(a, iter, val, val_prev, fcur, fbits, fsum);
    } else {
        if (inplace) k_pull_full<kSssp, kPullRows, true><<<full_blocks<kPullRows>(g), kBlock, 0, s>>>(a, iter, val, val_prev, fcur, fbits, fsum);
        else k_pull_full<kSssp, kPullRows><<<full_blocks<kPullRows>(g), kBlock, 0, s>>>(a, iter, val, val_prev, fcur, fbits, fsum);
    }
    return hipGetLastError();
}

template <int APP, int R, int FORM, bool INPLACE>
void launch_chunks_form(uint32_t blocks, const GraphArgs& a, uint32_t iter, int lc,
                        const uint32_t* list, const unsigned long long* mk, uint32_t* val,
                        const uint32_t* val_prev, const uint64_t* fcur, uint64_t* fbits,
                        uint32_t* fsum, hipStream_t s) {
    k_pull_chunks<APP, R, FORM, INPLACE><<<blocks, kBlock, 0, s>>>(a, iter, lc, list, mk, val, val_prev, fcur, fbits, fsum);
}

template <int APP, int R, bool INPLACE = false>
void launch_chunks_rows(uint64_t slots, const GraphArgs& a, uint32_t iter, int lc,
                        const uint32_t* list, const unsigned long long* mk, uint32_t* val,
                        const uint32_t* val_prev, const uint64_t* fcur, uint64_t* fbits,
                        uint32_t* fsum, hipStream_t s) {
    uint64_t waves = (slots + R - 1) / R;
    const uint64_t cap = 256ull * 32;  // resident waves on 256 CUs at 8 waves/SIMD
    if (waves > cap) waves = cap;
    const uint32_t blocks = (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    const int form = slot_form<R>(lc);
    if (form == kSlotsShared) launch_chunks_form<APP, R, kSlotsShared, INPLACE>(blocks, a, iter, lc, list, mk, val, val_prev, fcur, fbits, fsum, s);
    else if (form == kSlotsLong) launch_chunks_form<APP, R, kSlotsLong, INPLACE>(blocks, a, iter, lc, list, mk, val, val_prev, fcur, fbits, fsum, s);
    else launch_chunks_form<APP, R, kSlotsEach, INPLACE>(blocks, a, iter, lc, list, mk, val, val_prev, fcur, fbits, fsum, s);
}

hipError_t launch_pull_chunks(int app, const DevGraph& g, uint32_t iter, int log_chunk,
                              const uint32_t* list, const Ctl* ctl, uint64_t max_chunks,
                              uint32_t* val, const uint32_t* val_prev, const uint64_t* fcur,
                              uint64_t* fbits, uint32_t* fsum, hipStream_t s, int rows, bool inplace) {
    if (!max_chunks) return hipSuccess;
    if (app != kBfs && rows != kPullRows) return hipErrorInvalidValue;
    if (inplace && app == kBfs) return hipErrorInvalidValue;
    const uint64_t slots = log_chunk <= 6
                               ? (max_chunks + (64u >> log_chunk) - 1) / (64u >> log_chunk)
                               : max_chunks << (log_chunk - 6);
    GraphArgs a = args_of(g);
    const unsigned long long* mk = &ctl->marked;
    if (app == kBfs) {
        switch (rows) {
            case 4: launch_chunks_rows<kBfs, 4>(slots, a, iter, log_chunk, list, mk, val, val_prev, fcur, fbits, fsum, s); break;
            case 16: launch_chunks_rows<kBfs, 16>(slots, a, iter, log_chunk, list, mk, val, val_prev, fcur, fbits, fsum, s); break;
            case kPullRows: launch_chunks_rows<kBfs, kPullRows>(slots, a, iter, log_chunk, list, mk, val, val_prev, fcur, fbits, fsum, s); break;
            default: return hipErrorInvalidValue;
        }
    } else if (app == kCc) {
        if (inplace) launch_chunks_rows<kCc, kPullRows, true>(slots, a, iter, log_chunk, list, mk, val, val_prev, fcur, fbits, fsum, s);
        else launch_chunks_rows<kCc, kPullRows>(slots, a, iter, log_chunk, list, mk, val, val_prev, fcur, fbits, fsum, s);
    } else {
        if (inplace) launch_chunks_rows<kSssp, kPullRows, true>(slots, a, iter, log_chunk, list, mk, val, val_prev, fcur, fbits, fsum, s);
        else launch_chunks_rows<kSssp, kPullRows>(slots, a, iter, log_chunk, list, mk, val, val_prev, fcur, fbits, fsum, s);
    }
    return hipGetLastError();
}

hipError_t launch_pr_init(uint32_t n, const uint32_t* row_off, float* rank, float* contrib,
                          float* sum, hipStream_t s, uint32_t lg, uint64_t cap) {
    if (!n) return hipSuccess;
    k_pr_init<<<grid_for(n, 8192), kBlock, 0, s>>>(n, row_off, rank, contrib, sum, lg, cap);
    return hipGetLastError();
}

hipError_t launch_pr_pull(const DevGraph& g, const float* contrib, float* sum, float* head,
                          float* tail, int cus, hipStream_t s) {
    if (!g.rows) return hipSuccess;
    if (g.xs_rows) {
        // one launch per source slice, each over the whole GPU (resident blocks
        // at the full LDS size), adding into S; head/tail are indexed by the
        // sliced copy's tiles (no tile straddles two slices)
        constexpr size_t lds = (kHotVerts + 8) * sizeof(float);
        const int per_cu = g.xs_packed ? resident_blocks<k_pr_pull_slice<kPrTileRows, true>>(kHotBlock, lds)
                                       : resident_blocks<k_pr_pull_slice<kPrTileRows, false>>(kHotBlock, lds);
        if (per_cu <= 0) return hipErrorInvalidConfiguration;
        for (int j = 0; j < (1 << g.xs_lg); ++j) {
            const uint64_t rb = g.xs_row_begin[j], re = g.xs_row_begin[j + 1];
            if (re == rb) continue;
            GraphArgs xa = xs_args_of(g);
            xa.m = g.xs_edge_end[j];  // positions past the slice's last in-edge are idle
            xa.rows = (uint32_t)re;
            const uint32_t hot = slice_hot_count(g.n, (uint32_t)j, g.xs_lg);
            const uint64_t tb = rb / kPrTileRows, te = re / kPrTileRows;
            const uint64_t blocks = std::min<uint64_t>((uint64_t)std::max(cus, 1) * (uint64_t)per_cu,
                                                       (te - tb + kHotBlock / 64 - 1) / (kHotBlock / 64));
            // contributions are slice-major (see xs_contrib_cap)
            const float* cs = contrib + (uint64_t)j * xs_contrib_cap(g);
            if (g.xs_packed)
                k_pr_pull_slice<kPrTileRows, true><<<(uint32_t)blocks, kHotBlock, lds, s>>>(
                    xa, g.xs_lg, tb, te, cs, sum, head, tail, hot);
            else
                k_pr_pull_slice<kPrTileRows, false><<<(uint32_t)blocks, kHotBlock, lds, s>>>(
                    xa, g.xs_lg, tb, te, cs, sum, head, tail, hot);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const uint64_t tiles = (g.rows + kPrTileRows - 1) / kPrTileRows;
    const uint32_t hot = std::min<uint32_t>(g.n, kHotVerts);
    if (cus > 0 && hot >= kHotMinVerts) {
        // resident blocks per CU at the full LDS size (the same for every graph)
        // (a function-local static: initialised once, safely across threads; a
        // failed query leaves 0, which selects the plain kernel)
        static const int per_cu = [] {
            int b = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_pr_pull_hot<kPrTileRows>, kHotBlock,
                                                             (kHotVerts + 8) * sizeof(float)) != hipSuccess) {
                (void)hipGetLastError();
                return 0;
            }
            return b;
        }();
        const uint64_t blocks = (uint64_t)cus * (uint64_t)per_cu;
        // the LDS copy pays off once every wave has several tiles to stride over
        if (per_cu > 0 && tiles >= 4 * blocks * (kHotBlock / 64)) {
            k_pr_pull_hot<kPrTileRows><<<(uint32_t)blocks, kHotBlock, (hot + 8) * sizeof(float), s>>>(
                args_of(g), contrib, sum, head, tail, hot, tiles);
            return hipGetLastError();
        }
    }
    const uint32_t blocks = (uint32_t)((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
    k_pr_pull<kPrTileRows><<<blocks, kBlock, 0, s>>>(args_of(g), contrib, sum, head, tail);
    return hipGetLastError();
}

hipError_t launch_pr_fixup(const DevGraph& g, const float* head, const float* tail, float* sum,
                           const double* partials, uint32_t parts, double* d_next, hipStream_t s) {
    if (g.xs_rows) {
        const uint64_t ns = g.xs_pspan_short, nl = g.xs_pspans - g.xs_pspan_short;
        if (ns) {
            k_pr_fixup_xs_short<<<(uint32_t)((ns + kBlock - 1) / kBlock), kBlock, 0, s>>>(
                g.xs_pspan_v, g.xs_pspan_off, g.xs_pspan_tt, ns, head, tail, sum);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        const uint32_t blocks = (uint32_t)((nl + kWavesPerBlock - 1) / kWavesPerBlock) + 1;
        k_pr_fixup_xs_long<<<blocks, kBlock, 0, s>>>(g.xs_pspan_v, g.xs_pspan_off, g.xs_pspan_tt, ns, nl,
                                                     head, tail, sum, partials, parts, d_next);
        return hipGetLastError();
    }
    const uint64_t ns = g.short_spans, nl = g.nspans - g.short_spans;
    if (ns) {
        k_pr_fixup_short<<<(uint32_t)((ns + kBlock - 1) / kBlock), kBlock, 0, s>>>(g.spans, ns, head, tail, sum);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const uint32_t blocks = (uint32_t)((nl + kWavesPerBlock - 1) / kWavesPerBlock) + 1;
    k_pr_fixup_long<<<blocks, kBlock, 0, s>>>(g.spans + 3 * ns, nl, head, tail, sum, partials, parts,
                                              d_next);
    return hipGetLastError();
}

uint32_t pr_epilogue_blocks(uint32_t n) {
    uint32_t b = (n + kPrEpilogueVerts - 1) / kPrEpilogueVerts;
    return b ? b : 1;
}

hipError_t launch_pr_epilogue(uint32_t n, const uint32_t* row_off, float* sum,
                              double damping, const double* d_cur, float* rank, float* contrib,
                              double* partials, uint32_t parts, hipStream_t s, uint32_t lg,
                              uint64_t cap) {
    if (!n) return hipSuccess;
    k_pr_epilogue<<<parts, kBlock, 0, s>>>(n, kPrEpilogueVerts, row_off, sum, damping, d_cur, rank,
                                           contrib, partials, lg, cap);
    return hipGetLastError();
}

hipError_t launch_set_f64(double* p, double v, hipStream_t s) {
    k_set_f64<<<1, 64, 0, s>>>(p, v);
    return hipGetLastError();
}

WEDGE_DEBUG_ACCESSOR(debug_take_kernels)

}  // namespace wedge
