// Device-side helpers shared by the HIP translation units (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "wedge_internal.h"

namespace wedge {
namespace dev {

constexpr int kBlock = 256;           // 4 waves
constexpr int kWavesPerBlock = kBlock / 64;
// LDS copy of the highest-out-degree vertices' values in the full pulls
#ifndef WEDGE_HOT_BLOCK
#define WEDGE_HOT_BLOCK 768
#endif
#ifndef WEDGE_HOT_VERTS
#define WEDGE_HOT_VERTS 16384
#endif
#ifndef WEDGE_HOT_BATCH
#define WEDGE_HOT_BATCH 8
#endif
constexpr int kHotBlock = WEDGE_HOT_BLOCK;          // threads per block
constexpr uint32_t kHotVerts = WEDGE_HOT_VERTS;     // values held in LDS (4 B each)
constexpr int kHotBatch = WEDGE_HOT_BATCH;          // rows loaded at a time per wave
constexpr uint32_t kHotMinVerts = 4096;
// waves per block of the stand-alone compaction kernels: each block makes one
// output-range reservation (an atomic on one shared counter), so fewer,
// larger blocks contend less; 8 waves measured best at R-MAT scale 24
// (2: 57.7, 4: 61.5, 8: 63.6, 16: 63.3 GTEPS for the whole bench step)
#ifndef WEDGE_COMPACT_WAVES
#define WEDGE_COMPACT_WAVES 8
#endif
constexpr int kCompactWaves = WEDGE_COMPACT_WAVES;
// minimum resident waves per SIMD requested for the integer pulls (caps their
// registers so that many rows' loads stay in flight per compute unit)
#ifdef WEDGE_PULL_WAVES
#define WEDGE_PULL_OCCUPANCY __attribute__((amdgpu_waves_per_eu(WEDGE_PULL_WAVES)))
#else
#define WEDGE_PULL_OCCUPANCY
#endif
#ifdef WEDGE_CHUNK_WAVES
#define WEDGE_CHUNK_OCCUPANCY __attribute__((amdgpu_waves_per_eu(WEDGE_CHUNK_WAVES)))
#else
#define WEDGE_CHUNK_OCCUPANCY
#endif
constexpr int kTranslateEpt = 4;      // frontier out-edges per lane in the translation
constexpr int kCompactWords = 8;      // 64-bit bitmap words per wave in the compaction
constexpr uint32_t kPrEpilogueVerts = 8192;  // vertices per PageRank epilogue block

// Device checks of debug builds (WEDGE_DEBUG_CHECKS): a failed check ORs its
// code into the translation unit's error word, which the host reads after
// every run (WEDGE_DEBUG_ACCESSOR defines the reader). Release builds compile
// them away.
#ifdef WEDGE_DEBUG_CHECKS
static __device__ unsigned wedge_debug_word;
#define WEDGE_DCHECK(cond, code) \
    do { if (!(cond)) atomicOr(&::wedge::dev::wedge_debug_word, (unsigned)(code)); } while (0)
#define WEDGE_DEBUG_ACCESSOR(name)                                                   \
    hipError_t name(unsigned* word) {                                                \
        *word = 0;                                                                   \
        hipError_t e = hipMemcpyFromSymbol(word, HIP_SYMBOL(dev::wedge_debug_word),  \
                                           sizeof(unsigned), 0, hipMemcpyDeviceToHost); \
        if (e != hipSuccess || !*word) return e;                                     \
        const unsigned zero = 0;                                                     \
        return hipMemcpyToSymbol(HIP_SYMBOL(dev::wedge_debug_word), &zero, sizeof(unsigned), 0, \
                                 hipMemcpyHostToDevice);                             \
    }
#else
#define WEDGE_DCHECK(cond, code) do { } while (0)
#define WEDGE_DEBUG_ACCESSOR(name) \
    hipError_t name(unsigned* word) { *word = 0; return hipSuccess; }
#endif

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t mask_le(int l) { return l == 63 ? ~0ull : ((2ull << l) - 1ull); }
__device__ __forceinline__ uint64_t mask_lt(int l) { return (1ull << l) - 1ull; }

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) { return __builtin_nontemporal_load(p); }

// Lanes from `l` up to (excluding) the next segment head.
// Lane l's value in every lane, for a wave-uniform l (one v_readlane, where
// __shfl would compute addresses and go through the LDS crossbar).
__device__ __forceinline__ uint32_t lane_bcast(uint32_t x, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, l & 63);
}
__device__ __forceinline__ float lane_bcast(float x, int l) {
    return __builtin_bit_cast(float, (uint32_t)__builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l & 63));
}

// Lane l-1's value in lane l (lane 0 keeps its own), and lane l+1's in lane l
// (lane 63 keeps its own): DPP whole-wave shifts by one lane, one VALU
// instruction each.
__device__ __forceinline__ uint32_t lane_prev(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t lane_next(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x130, 0xf, 0xf, false);
}
template <typename T>
__device__ __forceinline__ T lane_next_t(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, lane_next(__builtin_bit_cast(uint32_t, v)));
    } else {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint64_t lo = lane_next((uint32_t)b), hi = lane_next((uint32_t)(b >> 32));
        return __builtin_bit_cast(T, lo | (hi << 32));
    }
}

// Integer minimum of 64-bit values (min<uint64_t> resolves to a double
// overload in device code, which costs a dozen FP64 instructions).
__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__device__ __forceinline__ int seg_span(uint64_t heads, int l) {
    uint64_t rest = l == 63 ? 0ull : (heads >> (l + 1));
    return rest ? (int)__builtin_ctzll(rest) + 1 : 64 - l;
}

// Lane l's bit of a wave-uniform mask as a per-lane condition (the mask is
// used as the lane mask of one v_cndmask; no per-lane shift).
__device__ __forceinline__ bool lane_bit(uint64_t mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

// Suffix-doubling reduction restricted to the lane's segment (segments start
// at the lanes set in `heads`, a wave-uniform mask with bit 0 set): on return
// the head lane of each segment holds the reduction of its whole segment,
// combined in a fixed tree order. At step o lane l takes lane l + o's partial
// exactly when l + o <= 63 and no segment starts in (l, l + o]; those lanes
// form the mask z, which the scalar unit doubles from step to step
// (z_2o = z_o & (z_o >> o)).
template <typename T, typename Op>
__device__ __forceinline__ T seg_reduce(T v, uint64_t heads, Op op) {
    uint64_t z = ~(heads >> 1) & (~0ull >> 1);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        // step 1 by a DPP shift (lane 63 takes nothing)
        const T w = o == 1 ? lane_next_t(v) : __shfl_down(v, o, 64);
        const T t = op(v, w);
        v = lane_bit(z) ? t : v;
        z &= z >> o;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum_tree(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Largest j in [L, H] with a[j] <= key, a non-decreasing and a[L] <= key;
// key is the same in every lane. Each step probes 64 points at once, so the
// search takes ceil(log64(H-L+1)) dependent loads.
__device__ __forceinline__ uint32_t wave_last_le(const uint32_t* __restrict__ a, uint32_t L,
                                                 uint32_t H, uint64_t key, int lane) {
    while (H - L >= 64) {
        const uint32_t step = (H - L + 63) / 64;
        const uint64_t probe = (uint64_t)L + (uint64_t)lane * step;
        const bool ok = probe <= H && a[probe] <= key;
        const int last = 63 - __clzll(__ballot(ok));
        L = L + (uint32_t)last * step;
        H = min(H, L + step - 1);
    }
    const uint64_t probe = (uint64_t)L + lane;
    const bool ok = probe <= H && a[probe] <= key;
    return L + (uint32_t)(63 - __clzll(__ballot(ok)));
}

__device__ __forceinline__ void set_bit(uint64_t* bits, uint32_t i) {
    atomicOr(reinterpret_cast<uint32_t*>(bits) + (i >> 5), 1u << (i & 31));
}

// Hierarchical bitmaps. A bitmap that a compaction lists (the next frontier,
// the Wedge Frontier) has a summary of one 32-bit flag per 4096 bits, the
// range one compaction block covers. Every writer of a bit also stores 1 into
// the flag of its range (a plain store: concurrent writers store the same
// value), so the compaction reads a flag and skips a range nobody touched,
// and its cost follows the touched ranges rather than the bitmap's length. A
// null summary means "scan everything".
constexpr int kSumShift = 12;  // log2 of the bits per summary flag
static_assert(kCompactWaves * kCompactWords * 64 == (1 << kSumShift),
              "one summary flag per compaction block");

__device__ __forceinline__ void mark_sum(uint32_t* sum, uint32_t bit) {
    if (sum) sum[bit >> kSumShift] = 1u;
}

__device__ __forceinline__ void set_bit_sum(uint64_t* bits, uint32_t* sum, uint32_t i) {
    set_bit(bits, i);
    mark_sum(sum, i);
}



// Frontier transformation work of one wave (see k_translate). The wave covers
// out-edges [base, base + 64*EPT) of the concatenated lists of the listed
// frontier vertices (each has at least one out-edge), one 64-edge row at a
// time. 64 consecutive edges lie in at most 64 consecutive list entries, so
// lane l holds entry j0 + l of a window (its out-degree prefix and CSR row
// start) and every lane finds the owner of its edge by a 6-step shuffle
// search of that window; the only per-edge global load is the edge index.
template <int EPT>
__device__ __forceinline__ void translate_wave(uint64_t wave, const uint32_t* __restrict__ flist,
                                               const uint32_t* __restrict__ degpre,
                                               uint32_t fcount, uint32_t active,
                                               const uint32_t* __restrict__ row_off,
                                               const uint32_t* __restrict__ pos, int lc,
                                               uint32_t* __restrict__ wbits32,
                                               uint32_t* __restrict__ wsum) {
    const int lane = lane_id();
    const uint64_t base = wave * 64ull * EPT;
    if (base >= active) return;
    const uint64_t end = umin64(base + 64ull * EPT, active);
    uint32_t j0 = wave_last_le(degpre, 0, fcount - 1, base, lane);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const uint64_t row = base + (uint64_t)i * 64;
        if (row >= end) break;
        const uint32_t jw = j0 + lane;
        const uint32_t dw = jw < fcount ? degpre[jw] : 0xFFFFFFFFu;
        const uint32_t rw = jw < fcount ? row_off[flist[jw]] : 0u;
        const uint64_t a = row + lane;
        const bool valid = a < end;
        int t = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const int cand = t + step;
            const uint32_t d = __shfl(dw, cand & 63, 64);
            if (cand < 64 && d <= a) t = cand;
        }
        uint32_t key = kInf, bit = 0;
        const uint32_t dt = __shfl(dw, t, 64);
        const uint32_t rt = __shfl(rw, t, 64);
#ifdef WEDGE_DEBUG_CHECKS
        {
            // the owner found for edge a holds it: prefix[t] <= a < prefix[t+1]
            const uint32_t dn = __shfl(dw, (t + 1) & 63, 64);
            if (valid) WEDGE_DCHECK(dt <= a && (t == 63 || a < (uint64_t)dn), kDbgTranslate);
        }
#endif
        if (valid) {
            const uint32_t q = rt + (uint32_t)(a - dt);
            const uint32_t c = pos[q] >> lc;
            key = c >> 5;
            bit = 1u << (c & 31);
        }
        // next row's window starts at the vertex holding edge row + 64: the one
        // holding edge row + 63, or the next one when that begins exactly there
        // (every listed vertex has at least one edge, so a window of 64 vertices
        // from there covers the whole next row)
        j0 += lane_bcast((uint32_t)t, 63);
        if (j0 + 1 < fcount && degpre[j0 + 1] <= row + 64) ++j0;
        const uint32_t prev = lane_prev(key);  // lane 0 is a head whatever it reads
        const bool head = lane == 0 || prev != key;
        const uint64_t heads = __ballot(head);
        bit = seg_reduce(bit, heads, [](uint32_t x, uint32_t y) { return x | y; });
        if (head && valid) {
            atomicOr(wbits32 + key, bit);
            if (wsum) wsum[key >> (kSumShift - 5)] = 1u;
        }
    }
}

// Bitmap compaction work of one (virtual) block (see k_bitmap_compact).
// For every set bit v < limit of a word, load_set(v) is read first (the
// reads of all the wave's words in flight together) and on_set(v, value)
// runs afterwards; on_old(v) runs for every set bit of the word copy_to held
// before it is overwritten (COPY only). A wave's loads are issued word-batch
// by word-batch, never one word at a time: bitmap words (and the words being
// replaced), then the out-degree bounds and load_set of every set bit.
//
// sum_bits / sum_copy (nullable; used only when a block covers exactly one
// summary flag's range) are the summaries of bits and copy_to: a block whose
// flags are both clear returns at once (nothing set, nothing to clear); a
// processed block clears its bits flag and hands it to copy_to's.
//
// FROMVAL: the set bits are not read from `bits` (which stays all-zero) but
// are the vertices v < limit with cmp_new[v] < cmp_old[v] (the vertices a
// synchronous CC/SSSP pull lowered) or, without cmp_old, with cmp_new[v] ==
// level (the vertices a BFS pull reached); load_set(v) is then cmp_new[v],
// read with them. Every block is processed, and copy_to's flag says whether
// any bit was set.
template <int WAVES, bool DEG, bool COPY, int G, bool FROMVAL = false, class LoadSet, class OnSet, class OnOld>
__device__ __forceinline__ void bitmap_compact_block_ex(
    uint64_t vblock, uint64_t* __restrict__ bits, uint64_t words, uint32_t limit,
    const uint32_t* __restrict__ row_off, uint32_t* __restrict__ list,
    uint32_t* __restrict__ degpre, unsigned long long* counter, unsigned long long* total,
    uint64_t* __restrict__ copy_to, uint32_t* __restrict__ sum_bits,
    uint32_t* __restrict__ sum_copy, LoadSet load_set, OnSet on_set, OnOld on_old,
    const uint32_t* __restrict__ cmp_new = nullptr, const uint32_t* __restrict__ cmp_old = nullptr,
    uint32_t level = 0) {
    __shared__ unsigned long long s_wave[WAVES];
    __shared__ unsigned long long s_all[WAVES];
    __shared__ unsigned long long s_base;
    // a block may run this for several virtual blocks in a row: wait until every
    // wave has read the previous call's shared values before they are rewritten
    __syncthreads();
    constexpr bool kSummed = WAVES * G * 64 == (1 << kSumShift);
    uint32_t fb = 1u;
    if (kSummed && sum_bits && !FROMVAL) {
        // block-uniform: every thread reads the same flags and leaves together
        fb = sum_bits[vblock];
        const uint32_t fc = (COPY && sum_copy) ? sum_copy[vblock] : 0u;
        if (!fb && !fc) return;
    }
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    const uint64_t w0 = (vblock * WAVES + wid) * G;
    uint64_t mk[G], lm[G], old[G], pre[G];
    uint32_t deg[G], r0[G], r1[G];
    uint64_t cnt = 0, all = 0, dsum = 0;
    uint32_t xn[G];
    if (FROMVAL) {
        uint32_t xo[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint64_t wc = w0 + g < words ? w0 + g : words - 1;
            const uint32_t v = (uint32_t)(wc * 64 + lane);
            const uint32_t vc = v < limit ? v : 0u;
            xn[g] = cmp_new[vc];
            xo[g] = cmp_old ? cmp_old[vc] : 0u;
            old[g] = COPY ? copy_to[wc] : 0ull;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            __asm__ volatile("" : "+v"(xn[g]));
            __asm__ volatile("" : "+v"(xo[g]));
            if (COPY) __asm__ volatile("" : "+v"(old[g]));
            const uint32_t v = (uint32_t)((w0 + g) * 64 + lane);
            const bool changed = cmp_old ? xn[g] < xo[g] : xn[g] == level;
            mk[g] = __ballot(w0 + g < words && v < limit && changed);
        }
    } else {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint64_t wi = w0 + g;
            const uint64_t wc = wi < words ? wi : words - 1;
            mk[g] = bits[wc];
            old[g] = COPY ? copy_to[wc] : 0ull;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            __asm__ volatile("" : "+v"(mk[g]));
            if (COPY) __asm__ volatile("" : "+v"(old[g]));
            mk[g] = w0 + g < words ? mk[g] : 0ull;
        }
    }
    // per set bit: out-degree bounds and the caller's value (a lane whose bit
    // is clear reads vertex 0's, which is then ignored)
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t v = (uint32_t)((w0 + g) * 64 + lane);
        const bool set = lane_bit(mk[g]) && v < limit;
        const uint32_t vs = set ? v : 0u;
        if (DEG) {
            r0[g] = row_off[vs];
            r1[g] = row_off[vs + 1];
        }
        pre[g] = FROMVAL ? xn[g] : load_set(vs);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (DEG) {
            __asm__ volatile("" : "+v"(r0[g]));
            __asm__ volatile("" : "+v"(r1[g]));
        }
        if (!FROMVAL) __asm__ volatile("" : "+v"(pre[g]));
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        lm[g] = mk[g];
        deg[g] = 0;
        if (mk[g]) {
            all += __popcll(mk[g]);
            if (DEG) {
                if (lane_bit(mk[g])) deg[g] = r1[g] - r0[g];
                // vertices without out-edges are counted but not listed
                lm[g] = __ballot(deg[g] != 0);
                dsum += wave_sum_tree(deg[g]);
            }
            cnt += __popcll(lm[g]);
        }
    }
    if (lane == 0) { s_wave[wid] = (cnt << kDegBits) | dsum; s_all[wid] = all; }
    __syncthreads();
    unsigned long long a = 0;  // set bits of the block (thread 0)
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < WAVES; ++i) { t += s_wave[i]; a += s_all[i]; }
        s_base = t ? atomicAdd(counter, t) : 0ull;
        if (total && a) atomicAdd(total, a);
    }
    __syncthreads();
    unsigned long long base = s_base;
    for (int i = 0; i < wid; ++i) base += s_wave[i];
    uint32_t cb = (uint32_t)(base >> kDegBits);
    uint64_t db = base & kDegMask;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint64_t wi = w0 + g;
        const uint32_t v = (uint32_t)(wi * 64 + lane);
        if (COPY && wi < words) {
            if (lane_bit(old[g]) && v < limit) on_old(v);
            if (lane == 0) copy_to[wi] = mk[g];
        }
        if (!mk[g]) continue;
        if (lane_bit(mk[g]) && v < limit) on_set(v, pre[g]);
        if (!FROMVAL && lane == 0) bits[wi] = 0ull;
        if (!lm[g]) continue;
        const bool act = lane_bit(lm[g]);
        const uint32_t rank = (uint32_t)__popcll(lm[g] & mask_lt(lane));
        uint32_t dex = 0, dtot = 0;
        if (DEG) {
            uint32_t inc = wave_incl_scan(deg[g], lane);
            dex = inc - deg[g];
            dtot = lane_bcast(inc, 63);
        }
        if (act && v < limit) {
            list[cb + rank] = v;
            if (DEG) degpre[cb + rank] = (uint32_t)(db + dex);
        }
        cb += (uint32_t)__popcll(lm[g]);
        db += dtot;
    }
    if (kSummed && threadIdx.x == 0) {
        if (sum_bits) sum_bits[vblock] = 0u;
        // copy_to now holds what bits held
        if (COPY && sum_copy) sum_copy[vblock] = FROMVAL ? (a != 0ull ? 1u : 0u) : fb;
    }
}

// Destinations of R positions per lane, every load issued before any is
// used. Positions must be valid (< m); lanes without an edge pass position 0
// and mask the result themselves. A guarded load (valid ? load : default)
// would become a branch per row, and the wait at each branch join would
// serialise the rows' memory round trips.
template <int R>
__device__ __forceinline__ void dst_of_rows(const GraphArgs& g, const uint32_t (&pc)[R],
                                            uint32_t (&dst)[R]) {
    uint64_t mk[R];
    uint32_t sg[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        mk[i] = g.rowmask[pc[i] >> 6];
        sg[i] = g.rowseg[pc[i] >> 6];
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
        dst[i] = g.nzdst[sg[i] + (uint32_t)__popcll(mk[i] & ~1ull & mask_le((int)(pc[i] & 63)))];
}

// Wave-uniform read of a table no kernel writes, through the constant address
// space: the compiler may then use a scalar load, and merges the reads of
// consecutive entries into a few wide ones waited for once. (A vector load of
// a uniform address is waited for before its value can move to a scalar
// register, one entry at a time.)
template <typename T>
__device__ __forceinline__ T ld_uniform(const T* p, uint64_t i) {
    typedef const __attribute__((address_space(4))) T ConstT;
    return ((ConstT*)p)[i];
}

// Row layout of the N rows r0 .. r0 + N - 1 (r0 wave-uniform, below the
// layout's row count): their masks and segment indices, and the mask of the
// row after them. The device arrays carry kRowPad rows of padding (mask 1,
// the last segment index), so rows past the layout need no clamp.
template <int N>
__device__ __forceinline__ void row_layout(const GraphArgs& g, uint64_t r0, uint64_t (&mk)[N + 1],
                                           uint32_t (&sg)[N]) {
    static_assert(N + 1 <= (int)kRowPad, "rows read past the layout stay in its padding");
#pragma unroll
    for (int i = 0; i <= N; ++i) mk[i] = ld_uniform(g.rowmask, r0 + (uint64_t)i);
#pragma unroll
    for (int i = 0; i < N; ++i) sg[i] = ld_uniform(g.rowseg, r0 + (uint64_t)i);
}

// Destination of this lane's position in a whole row with mask mk and segment
// index sg (the full pulls: lane l of the row holds position row * 64 + l):
// the lane's segment is counted with mbcnt over the wave-uniform mask. A row
// of the padding gives the last segment's destination (its lanes are masked
// by the caller).
__device__ __forceinline__ uint32_t dst_of_whole_row(const GraphArgs& g, uint64_t mk, uint32_t sg) {
    const uint64_t m1 = mk & ~1ull;
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m1 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m1, 0u));
    return g.nzdst[sg + below + (lane_bit(m1) ? 1u : 0u)];
}

// Next-frontier bits of one row: every destination segment whose head lane
// has `commit` set gets its bit, with one atomicOr per distinct bitmap word
// (consecutive destinations share words, so a row of 64 positions needs one
// or two atomics instead of one per destination). All lanes must call it.
__device__ __forceinline__ void set_bits_row(uint64_t* __restrict__ fbits, uint32_t* __restrict__ fsum,
                                             uint32_t dst, bool commit, uint64_t heads, int lane) {
    if (!__ballot(commit)) return;  // most rows of a late iteration change nothing
    const int hl = 63 - __clzll(heads & mask_le(lane));  // head lane of this lane's segment
    const bool c = __shfl((int)commit, hl, 64) != 0;
    const uint32_t key = c ? (dst >> 5) : kInf;
    const uint32_t bit = (c && lane == hl) ? (1u << (dst & 31)) : 0u;
    const uint32_t prev = lane_prev(key);  // lane 0 is a head whatever it reads
    const bool head = lane == 0 || prev != key;
    const uint64_t wheads = __ballot(head);
    const uint32_t orv = seg_reduce(bit, wheads, [](uint32_t a, uint32_t b) { return a | b; });
    if (head && key != kInf) {
        atomicOr(reinterpret_cast<uint32_t*>(fbits) + key, orv);
        if (fsum) fsum[key >> (kSumShift - 5)] = 1u;
    }
}

// ROWS: the R positions of each lane are the lanes of R consecutive rows
// starting at a row the wave owns alone (the full pull). Then a destination
// whose in-edges all lie in the wave is written by this wave only, and takes
// a plain store instead of a min-atomic; only the wave's first and last
// segments can be shared with the neighbouring waves.
// INPLACE (CC and SSSP): sources' values are gathered from val, the array
// this iteration lowers, instead of the committed copy val_prev (an
// asynchronous, Gauss-Seidel style pull: a value lowered earlier in the same
// iteration travels on at once). Every value read is still the length of a
// real path (or a real label), and values only fall, so the fixed point, and
// the final result, are those of the synchronous pull.
//
// Edges says how a pull reads an in-edge: the canonical arrays (a source id
// per position, SSSP weights in their own array), or the source-sliced copy,
// whose words may pack (slice-local source << 8) | weight and whose slice's
// highest-out-degree sources can have their values staged in LDS.
//
// BITS = false (full pulls): no next-frontier bits are set. CC and SSSP: at
// the start of an iteration val equals val_prev, the committed copy (the
// in-place pull keeps it too, only to compare against), and values only
// fall, so the vertices this pull lowers are exactly those with val <
// val_prev afterwards. BFS: the vertices this pull reaches are exactly those
// with val == iter + 1 afterwards (no earlier iteration wrote that level).
// The finalisation derives the bitmap from the values (one streaming pass)
// instead of every row building its bitmap words.
struct CanonicalEdges {
    static constexpr bool kPacked = false;
    __device__ __forceinline__ uint32_t gather(const uint32_t* __restrict__ src, uint32_t u) const {
        return src[u];
    }
    // 32-bit word wq of the current frontier bitmap (BFS)
    __device__ __forceinline__ uint32_t fword(const uint32_t* __restrict__ f, uint32_t wq) const {
        return f[wq];
    }
};

// BFS full pull with the frontier bitmap's first `words` 32-bit words (the
// bits of the lowest, highest-out-degree ids) copied into LDS.
struct HotFrontierEdges : CanonicalEdges {
    uint32_t words;
    const uint32_t* __restrict__ s_bits;  // LDS
    __device__ __forceinline__ uint32_t fword(const uint32_t* __restrict__ f, uint32_t wq) const {
        const bool h = wq < words;
        const uint32_t gv = f[h ? 0u : wq];
        const uint32_t lv = s_bits[h ? wq : 0u];
        return h ? lv : gv;
    }
};

template <bool PACKED, bool HOT>
struct SliceEdges {
    static constexpr bool kPacked = PACKED;
    uint32_t slice;
    uint32_t lg;                        // log2 of the number of slices
    uint32_t n;
    uint32_t hot;                       // values of slice-local ids [0, hot) are in s_hot
    const uint32_t* __restrict__ s_hot;  // LDS
    __device__ __forceinline__ uint32_t gather(const uint32_t* __restrict__ src, uint32_t word) const {
        const uint32_t l = PACKED ? (word >> 8) : xcd_slice_local(word, lg);
        uint32_t u = word;
        if (PACKED) {
            // a lane without an edge holds another slice's word: keep its
            // (masked) read inside the array
            u = xcd_slice_global(l, slice, lg);
            u = u < n ? u : 0u;
        }
        if (!HOT) return src[u];
        // branch-free: the lane's global and LDS reads are both issued
        const bool h = l < hot;
        const uint32_t gv = src[h ? 0u : u];
        const uint32_t lv = s_hot[h ? l : 0u];
        return h ? lv : gv;
    }
    __device__ __forceinline__ uint32_t fword(const uint32_t* __restrict__ f, uint32_t wq) const {
        return f[wq];  // BFS does not pull over the sliced copy
    }
};

template <int APP, int R, bool ROWS = false, bool INPLACE = false, class Edges = CanonicalEdges,
          bool BITS = true>
__device__ __forceinline__ void pull_lanes(const GraphArgs& g, const uint32_t (&p)[R],
                                           const bool (&valid)[R], uint32_t iter,
                                           uint32_t* __restrict__ val,
                                           const uint32_t* __restrict__ val_prev,
                                           const uint64_t* __restrict__ fcur,
                                           uint64_t* __restrict__ fbits,
                                           uint32_t* __restrict__ fsum,
                                           const Edges edges = Edges{}) {
    static_assert(ROWS || !Edges::kPacked, "the chunk pulls read the canonical arrays");
    const int lane = lane_id();
    // loads are branch-free: a lane without an edge reads position 0 (its
    // results are masked), so all rows' loads of one step are in flight at once
    uint32_t pc[R], dst[R], u[R], wt[R];
#pragma unroll
    for (int i = 0; i < R; ++i) pc[i] = valid[i] ? p[i] : 0u;
    // ROWS: the wave's rows are r0 .. r0 + R - 1. Their edge streams are read
    // at a wave-uniform row address plus the lane (the in-edge arrays extend
    // to whole rows: padded on the device, and the sliced copy by its layout)
    const uint64_t r0 = ROWS ? (uint32_t)__builtin_amdgcn_readfirstlane((int)p[0]) >> 6 : 0u;
    if (APP != kBfs) {
        // the edge streams do not depend on the destinations: issue them first
#pragma unroll
        for (int i = 0; i < R; ++i)
            u[i] = ld_stream(ROWS ? g.in_src + ((r0 + i) << 6) + lane : g.in_src + pc[i]);
#pragma unroll
        for (int i = 0; i < R; ++i)
            wt[i] = APP == kSssp ? (Edges::kPacked ? (u[i] & 255u)
                                                   : ld_stream(ROWS ? g.in_w + ((r0 + i) << 6) + lane
                                                                    : g.in_w + pc[i]))
                                 : 0u;
    }
    // ROWS: the rows' layout is read once
    uint64_t rmk[R + 1];
    uint32_t rsg[R];
    if constexpr (ROWS) {
        row_layout<R>(g, r0, rmk, rsg);
#pragma unroll
        for (int i = 0; i < R; ++i) dst[i] = dst_of_whole_row(g, rmk[i], rsg[i]);
    } else {
        dst_of_rows<R>(g, pc, dst);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) dst[i] = valid[i] ? dst[i] : kInf;
#ifdef WEDGE_DEBUG_CHECKS
#pragma unroll
    for (int i = 0; i < R; ++i) {
        if (!valid[i]) continue;
        WEDGE_DCHECK(pc[i] < g.m, kDbgPullPos);
        WEDGE_DCHECK(dst[i] < g.n, kDbgPullDst);
        if (dst[i] < g.n && g.col_off)
            WEDGE_DCHECK(g.col_off[dst[i]] <= pc[i] && pc[i] < g.col_off[dst[i] + 1], kDbgPullEdge);
    }
#endif

    if (APP == kBfs) {
        // only unvisited destinations read their in-edges: the others point
        // their loads at one shared address (one request per wave)
        bool need[R];
        uint32_t vd[R];
#pragma unroll
        for (int i = 0; i < R; ++i) vd[i] = val[valid[i] ? dst[i] : 0u];
#pragma unroll
        for (int i = 0; i < R; ++i) need[i] = valid[i] & (vd[i] == kInf);
#pragma unroll
        for (int i = 0; i < R; ++i) u[i] = ld_stream(g.in_src + (need[i] ? pc[i] : 0u));
        uint32_t fw[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint32_t q = need[i] ? u[i] : 0u;
            fw[i] = edges.fword(reinterpret_cast<const uint32_t*>(fcur), q >> 5) >> (q & 31);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) need[i] = need[i] & ((fw[i] & 1u) != 0u);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const bool found = need[i];
            uint64_t heads;
            bool head;
            if constexpr (ROWS) {
                // segment starts are the row's mask bits (consecutive segments
                // have distinct destinations); every lane without an edge
                // forms a segment of its own
                heads = rmk[i] | 1ull | ~__ballot(valid[i]);
                head = lane_bit(heads);
            } else {
                const uint32_t prev = lane_prev(dst[i]);  // lane 0 is a head whatever it reads
                head = lane == 0 || prev != dst[i];
                heads = __ballot(head);
            }
            const uint64_t fm = __ballot(found);
            bool commit = false;
            if (head && dst[i] != kInf) {
                const int span = seg_span(heads, lane);
                const uint64_t seg = span >= 64 ? ~0ull : ((1ull << span) - 1ull);
                commit = ((fm >> lane) & seg) != 0;
                if (commit) val[dst[i]] = iter + 1;
            }
            if (BITS) set_bits_row(fbits, fsum, dst[i], commit, heads, lane);
        }
    } else {
        // All loads of the R rows are issued before any result is used, and
        // the commit waits for nothing: within an iteration val[v] only falls
        // from val_prev[v], so best < (any value of val[v] read now) already
        // proves that v changes this iteration and belongs to the next
        // frontier, whatever the min-atomic finds when it lands. A destination
        // whose segment runs on into the next row is carried there, so each
        // destination is committed at most once per wave (a hub spanning many
        // rows would otherwise send one atomic per row to the same address).
        uint32_t x[R], cur[R];
        if (!ROWS) {
            // Pull over marked chunks: most sources of a marked chunk are
            // inactive, so test the source's frontier bit (a 1-bit gather from
            // an L2-resident bitmap) and gather the value of active sources
            // only; inactive ones read one shared address. Any superset of the
            // active edges gives the same result (reading 1). The full pull
            // gathers without the test: there most sources are active and the
            // bit only adds a dependent load.
            uint32_t fw[R];
#pragma unroll
            for (int i = 0; i < R; ++i) fw[i] = reinterpret_cast<const uint32_t*>(fcur)[u[i] >> 5];
#pragma unroll
            for (int i = 0; i < R; ++i) cur[i] = val[valid[i] ? dst[i] : 0u];
            bool act[R];
#pragma unroll
            for (int i = 0; i < R; ++i) act[i] = valid[i] & (((fw[i] >> (u[i] & 31)) & 1u) != 0u);
#pragma unroll
            for (int i = 0; i < R; ++i) x[i] = (INPLACE ? val : val_prev)[act[i] ? u[i] : 0u];
#pragma unroll
            for (int i = 0; i < R; ++i) x[i] = act[i] ? x[i] : kInf;
        } else {
#pragma unroll
            for (int i = 0; i < R; ++i) x[i] = edges.gather(INPLACE ? val : val_prev, u[i]);
#pragma unroll
            for (int i = 0; i < R; ++i) cur[i] = val[valid[i] ? dst[i] : 0u];
#pragma unroll
            for (int i = 0; i < R; ++i) x[i] = valid[i] ? x[i] : kInf;
        }
        uint32_t carry = kInf;
        bool first_shared = true, last_shared = true, lane0_first = true;
        if constexpr (ROWS) {
            // the row after the wave's rows is in the layout's padding (mask 1)
            // when the wave holds the last rows
            first_shared = !(rmk[0] & 1ull);
            last_shared = !(rmk[R] & 1ull);
        }
        // ROWS: the segment starts of a row are its mask bits (consecutive
        // segments have distinct destinations), and every lane without an
        // edge forms a segment of its own. The rows' reductions are
        // independent of each other and of the commits: they run first, in
        // one branch-free block, so that their dependent cross-lane steps
        // overlap instead of waiting for each row's commit branches.
        uint32_t red[R];
        if constexpr (ROWS) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                // an unreached source (kInf) stays kInf; a reached one's sum
                // does not overflow ((n - 1) * max weight < kInf)
                const uint32_t cand = APP == kCc ? x[i] : __builtin_elementwise_add_sat(x[i], wt[i]);
                red[i] = seg_reduce(cand, rmk[i] | 1ull | ~__ballot(valid[i]),
                                    [](uint32_t a, uint32_t b) { return a < b ? a : b; });
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            uint64_t heads;
            bool head;
            uint32_t best;
            if constexpr (ROWS) {
                heads = rmk[i] | 1ull | ~__ballot(valid[i]);  // as in the BFS branch
                head = lane_bit(heads);
                best = red[i];
            } else {
                const uint32_t cand = APP == kCc ? x[i] : __builtin_elementwise_add_sat(x[i], wt[i]);
                const uint32_t prev = lane_prev(dst[i]);  // lane 0 is a head whatever it reads
                head = lane == 0 || prev != dst[i];
                heads = __ballot(head);
                best = seg_reduce(cand, heads, [](uint32_t a, uint32_t b) { return a < b ? a : b; });
            }
            const uint64_t hv = heads & __ballot(valid[i]);
            if (lane == 0 && carry < best) best = carry;
            carry = kInf;
            int defer = -1;
            const int h_last = hv ? 63 - __clzll(hv) : -1;
            bool commit;
            if constexpr (ROWS) {
                // the last segment runs on into the next row when that row's
                // lane 0 holds an edge and starts no segment (then every lane
                // of this row holds one, so the segment is h_last's); which
                // lanes commit, and which of those share their destination
                // with a neighbouring wave, are wave-uniform masks
                if (hv && i + 1 < R && !(rmk[i + 1] & 1ull) && (__ballot(valid[i + 1]) & 1ull)) {
                    defer = h_last;
                    carry = lane_bcast(best, h_last);
                }
                const uint64_t cm = defer >= 0 ? hv & ~(1ull << defer) : hv;
                const uint64_t sm = ((lane0_first && first_shared) ? 1ull : 0ull) |
                                    ((i == R - 1 && last_shared && h_last >= 0) ? (1ull << h_last) : 0ull);
                commit = lane_bit(cm) && best < cur[i];
                if (commit) {
                    if (lane_bit(sm)) atomicMin(val + dst[i], best);
                    else val[dst[i]] = best;
                }
            } else {
                if (hv && i + 1 < R) {
                    if (lane_bcast(dst[i + 1], 0) == lane_bcast(dst[i], h_last)) {
                        defer = h_last;
                        carry = lane_bcast(best, h_last);
                    }
                }
                commit = head && valid[i] && lane != defer && best < cur[i];
                if (commit) atomicMin(val + dst[i], best);
            }
            if (BITS) set_bits_row(fbits, fsum, dst[i], commit, heads, lane);
            lane0_first = lane0_first && defer == 0;
        }
    }
}

// FROMVAL: the set bits are the vertices with val < val_prev (COMMIT) or
// with val == level (BFS, without COMMIT).
template <bool DEG, bool COMMIT, bool COPY, int G, int WAVES = kWavesPerBlock, bool FROMVAL = false>
__device__ __forceinline__ void bitmap_compact_block(
    uint64_t vblock, uint64_t* __restrict__ bits, uint64_t words, uint32_t limit,
    const uint32_t* __restrict__ row_off, uint32_t* __restrict__ list,
    uint32_t* __restrict__ degpre, unsigned long long* counter, unsigned long long* total,
    uint32_t* __restrict__ val_prev, const uint32_t* __restrict__ val,
    uint64_t* __restrict__ copy_to, uint32_t* __restrict__ sum_bits = nullptr,
    uint32_t* __restrict__ sum_copy = nullptr, uint32_t level = 0) {
    bitmap_compact_block_ex<WAVES, DEG, COPY, G, FROMVAL>(
        vblock, bits, words, limit, row_off, list, degpre, counter, total, copy_to, sum_bits, sum_copy,
        [&](uint32_t v) -> uint64_t { return COMMIT ? val[v] : 0u; },
        [&](uint32_t v, uint64_t x) { if (COMMIT) val_prev[v] = (uint32_t)x; }, [](uint32_t) {},
        FROMVAL ? val : nullptr, (FROMVAL && COMMIT) ? val_prev : nullptr, level);
}

// Positions covered by lane `lane` of the chunk-list slots s0 .. s0+R-1: a
// slot is 64 lanes over 64 >> lc chunks (lc <= 6) or one 64-position part of
// a chunk (lc > 6). Lanes past the `slots` slots or the K >= 1 listed chunks
// get valid = false. When the R slots cover at most 64 consecutive list
// entries (chunks of 8 or more edges), the wave reads them with one
// coalesced load and every lane takes its entry by a shuffle; otherwise each
// slot reads its own entries. Positions are 32-bit, so slot and chunk
// indices are too. FORM (see slot_form) picks one of the three cases at
// compile time, so a kernel carries the registers of one case only.
enum SlotForm : int { kSlotsShared = 0, kSlotsLong = 1, kSlotsEach = 2 };

template <int R>
__host__ __device__ constexpr int slot_form(int lc) {
    return lc > 6 ? kSlotsLong : ((R << (6 - lc)) <= 64 ? kSlotsShared : kSlotsEach);
}

template <int R, int FORM>
__device__ __forceinline__ void chunk_slot_rows(uint64_t s0w, uint64_t slotsw, int lane, int lc,
                                                const uint32_t* __restrict__ list, uint64_t Kw,
                                                uint64_t m, uint32_t (&p)[R], bool (&valid)[R]) {
    const uint32_t s0 = (uint32_t)s0w, slots = (uint32_t)slotsw, K = (uint32_t)Kw;
    const uint32_t ul = (uint32_t)lane;
    if (FORM == kSlotsShared) {
        const uint32_t per = 64u >> lc;
        const uint32_t first = s0 * per;
        const uint32_t e = first + ul;
        const uint32_t mine = list[e < K ? e : K - 1];
        const uint32_t sub = ul >> lc;
        const uint32_t off = ul & ((1u << lc) - 1u);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint32_t idx = (uint32_t)i * per + sub;
            const uint32_t c = __shfl(mine, (int)idx, 64);
            const uint64_t pp = ((uint64_t)c << lc) + off;
            // a listed chunk starts inside the in-edge array
            WEDGE_DCHECK(!((s0 + i < slots) & (first + idx < K)) || ((uint64_t)c << lc) < m, kDbgChunk);
            valid[i] = (s0 + i < slots) & (first + idx < K) & (pp < m);
            p[i] = valid[i] ? (uint32_t)pp : 0u;
        }
    } else if (FORM == kSlotsLong) {
        const int hi = lc - 6;
        const uint32_t first = s0 >> hi;
        const uint32_t e = first + ul;
        const uint32_t mine = list[e < K ? e : K - 1];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint32_t s = s0 + (uint32_t)i;
            const uint32_t idx = (s >> hi) - first;
            const uint32_t c = __shfl(mine, (int)idx, 64);
            const uint64_t pp = ((uint64_t)c << lc) + ((uint64_t)(s & ((1u << hi) - 1u)) << 6) + ul;
            WEDGE_DCHECK(!((s < slots) & (first + idx < K)) || ((uint64_t)c << lc) < m, kDbgChunk);
            valid[i] = (s < slots) & (first + idx < K) & (pp < m);
            p[i] = valid[i] ? (uint32_t)pp : 0u;
        }
    } else {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            uint64_t pp = ~0ull;
            if (s0 + i < slots) {
                const uint32_t ci = (s0 + (uint32_t)i) * (64u >> lc) + (ul >> lc);
                const uint32_t off = ul & ((1u << lc) - 1u);
                if (ci < K) {
                    pp = ((uint64_t)list[ci] << lc) + off;
                    WEDGE_DCHECK(((uint64_t)list[ci] << lc) < m, kDbgChunk);
                }
            }
            valid[i] = pp < m;
            p[i] = valid[i] ? (uint32_t)pp : 0u;
        }
    }
}

// The same with the case chosen at run time (kernels that serve every group
// size from one instantiation).
template <int R>
__device__ __forceinline__ void chunk_slot_rows_any(uint64_t s0, uint64_t slots, int lane, int lc,
                                                    const uint32_t* __restrict__ list, uint64_t K,
                                                    uint64_t m, uint32_t (&p)[R], bool (&valid)[R]) {
    const int form = slot_form<R>(lc);
    if (form == kSlotsShared) chunk_slot_rows<R, kSlotsShared>(s0, slots, lane, lc, list, K, m, p, valid);
    else if (form == kSlotsLong) chunk_slot_rows<R, kSlotsLong>(s0, slots, lane, lc, list, K, m, p, valid);
    else chunk_slot_rows<R, kSlotsEach>(s0, slots, lane, lc, list, K, m, p, valid);
}

__device__ __forceinline__ uint64_t chunk_slots(uint64_t K, int lc) { return chunk_slots_count(K, lc); }

}  // namespace dev
}  // namespace wedge
