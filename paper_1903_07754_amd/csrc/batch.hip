// Batched BFS on gfx950: many sources as 64-bit masks, many graphs as one
// disjoint union, and a persistent kernel that runs a whole traversal in one
// launch.
//
// Multi-source BFS follows the bit-parallel formulation of Then et al. ("The
// More the Merrier", PVLDB 8(4), 2014) on top of the Wedge pull: vertex v
// keeps visited[v], cur[v] and nxt[v] as 64-bit masks (bit s = source s), and
// one pull sets nxt[v] |= OR over in-edges of cur[u], minus visited[v]. The
// vertex frontier the Wedge machinery sees is {v : cur[v] != 0}, so gating,
// translation and compaction are exactly those of single-source BFS.
#include "device_common.h"

namespace wedge {
namespace {

using namespace dev;

// ------------------------------------------------------------ pull (masks)
template <int R>
__device__ __forceinline__ void ms_pull_lanes(const GraphArgs& g, const uint32_t (&p)[R],
                                              const bool (&valid)[R], uint64_t all,
                                              const uint64_t* __restrict__ visited,
                                              const uint64_t* __restrict__ cur,
                                              uint64_t* __restrict__ nxt,
                                              uint64_t* __restrict__ fbits,
                                              uint32_t* __restrict__ fsum) {
    const int lane = lane_id();
    // branch-free loads (see pull_lanes): lanes without an edge read position
    // 0, lanes that need no edge point at one shared address, and loaded
    // values are pinned so the loads are not turned back into branches
    uint32_t pc[R], dst[R], u[R];
    uint64_t vis[R], x[R];
    bool need[R];
#pragma unroll
    for (int i = 0; i < R; ++i) pc[i] = valid[i] ? p[i] : 0u;
    dst_of_rows<R>(g, pc, dst);
#pragma unroll
    for (int i = 0; i < R; ++i) dst[i] = valid[i] ? dst[i] : kInf;
#pragma unroll
    for (int i = 0; i < R; ++i) vis[i] = visited[valid[i] ? dst[i] : 0u];
#pragma unroll
    for (int i = 0; i < R; ++i) __asm__ volatile("" : "+v"(vis[i]));
#pragma unroll
    for (int i = 0; i < R; ++i) {
        vis[i] = valid[i] ? vis[i] : all;
        need[i] = (vis[i] & all) != all;  // a destination seen by every source is skipped
    }
#pragma unroll
    for (int i = 0; i < R; ++i) u[i] = ld_stream(g.in_src + (need[i] ? pc[i] : 0u));
#pragma unroll
    for (int i = 0; i < R; ++i) __asm__ volatile("" : "+v"(u[i]));
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = cur[need[i] ? u[i] : 0u];
#pragma unroll
    for (int i = 0; i < R; ++i) __asm__ volatile("" : "+v"(x[i]));
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = need[i] ? x[i] : 0ull;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t prev = lane_prev(dst[i]);  // lane 0 is a head whatever it reads
        const bool head = lane == 0 || prev != dst[i];
        const uint64_t heads = __ballot(head);
        const uint64_t orv = seg_reduce(x[i], heads,
                                        [](uint64_t a, uint64_t b) { return a | b; });
        if (head && dst[i] != kInf) {
            const uint64_t nb = orv & ~vis[i] & all;
            if (nb) {
                atomicOr(reinterpret_cast<unsigned long long*>(nxt + dst[i]),
                         (unsigned long long)nb);
                set_bit_sum(fbits, fsum, dst[i]);
            }
        }
    }
}

template <int R>
__device__ __forceinline__ void ms_pull_rows(const GraphArgs& g, uint64_t r0, uint64_t all,
                                             const uint64_t* visited, const uint64_t* cur,
                                             uint64_t* nxt, uint64_t* fbits, uint32_t* fsum) {
    const int lane = lane_id();
    uint32_t p[R];
    bool valid[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint64_t pp = (r0 + i) * 64 + lane;
        valid[i] = pp < g.m;
        p[i] = (uint32_t)pp;
    }
    ms_pull_lanes<R>(g, p, valid, all, visited, cur, nxt, fbits, fsum);
}

template <int R>
__device__ __forceinline__ void ms_pull_slots(const GraphArgs& g, uint64_t s0, uint64_t slots,
                                              int lc, const uint32_t* list, uint64_t K,
                                              uint64_t all, const uint64_t* visited,
                                              const uint64_t* cur, uint64_t* nxt,
                                              uint64_t* fbits, uint32_t* fsum) {
    const int lane = lane_id();
    uint32_t p[R];
    bool valid[R];
    chunk_slot_rows_any<R>(s0, slots, lane, lc, list, K, g.m, p, valid);
    ms_pull_lanes<R>(g, p, valid, all, visited, cur, nxt, fbits, fsum);
}

// Commit of one multi-source iteration, over the next-frontier bitmap: list the
// vertices (with out-degree prefix), add the new masks to visited, write level
// `level` for every newly set (vertex, source) bit into lev[v*K + s], clear
// the masks of the frontier being retired, and move the bitmap to fcur.
template <int WAVES = kWavesPerBlock>
__device__ __forceinline__ void ms_finalize_block(
    uint64_t vblock, uint64_t* bits, uint64_t words, uint32_t n, const uint32_t* row_off,
    uint32_t* list, uint32_t* degpre, Ctl* ctl, uint64_t* fcur, uint64_t* visited,
    uint64_t* retire, const uint64_t* nxt, uint32_t* lev, uint32_t K, uint32_t level,
    uint32_t* fsum = nullptr, uint32_t* csum = nullptr) {
    // the new masks of the wave's vertices, one slot per (word, lane), for the
    // level writes below (each lane only touches its own slots)
    __shared__ uint64_t s_nb[WAVES][kCompactWords][64];
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int g = 0; g < kCompactWords; ++g) s_nb[wid][g][lane] = 0ull;
    bitmap_compact_block_ex<WAVES, true, true, kCompactWords>(
        vblock, bits, words, n, row_off, list, degpre, &ctl->fnext, &ctl->ftotal, fcur, fsum, csum,
        [&](uint32_t v) -> uint64_t { return nxt[v]; },
        [&](uint32_t v, uint64_t nb) {
            atomicOr(reinterpret_cast<unsigned long long*>(visited + v), (unsigned long long)nb);
            s_nb[wid][(v >> 6) % kCompactWords][lane] = nb;
        },
        [&](uint32_t v) { retire[v] = 0ull; });
    // levels: one coalesced store of a vertex's row (lane s writes source s)
    // per newly reached vertex, instead of one scattered store per new bit
    const uint64_t w0 = (vblock * WAVES + wid) * kCompactWords;
#pragma unroll
    for (int g = 0; g < kCompactWords; ++g) {
        const uint64_t nbv = s_nb[wid][g][lane];
        uint64_t todo = __ballot(nbv != 0ull);
        while (todo) {
            const int j = __builtin_ctzll(todo);
            todo &= todo - 1;
            const uint64_t nb = __shfl(nbv, j, 64);
            const uint64_t v = (w0 + g) * 64 + (uint64_t)j;
            if ((uint32_t)lane < K && ((nb >> lane) & 1ull)) lev[v * K + lane] = level;
        }
    }
}

template <int WAVES = kWavesPerBlock>
__device__ __forceinline__ void bfs_finalize_block(uint64_t vblock, uint64_t* bits,
                                                   uint64_t words, uint32_t n,
                                                   const uint32_t* row_off, uint32_t* list,
                                                   uint32_t* degpre, Ctl* ctl, uint64_t* fcur) {
    bitmap_compact_block_ex<WAVES, true, true, kCompactWords>(
        vblock, bits, words, n, row_off, list, degpre, &ctl->fnext, &ctl->ftotal, fcur, nullptr, nullptr,
        [](uint32_t) -> uint64_t { return 0ull; }, [](uint32_t, uint64_t) {}, [](uint32_t) {});
}

// --------------------------------------------------- per-iteration kernels

template <int R>
__global__ __launch_bounds__(kBlock) void k_ms_pull_full(GraphArgs g, uint64_t all,
                                                         const uint64_t* __restrict__ visited,
                                                         const uint64_t* __restrict__ cur,
                                                         uint64_t* __restrict__ nxt,
                                                         uint64_t* __restrict__ fbits,
                                                         uint32_t* __restrict__ fsum) {
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t r0 = wave * R;
    if (r0 >= g.rows) return;
    ms_pull_rows<R>(g, r0, all, visited, cur, nxt, fbits, fsum);
}

template <int R>
__global__ __launch_bounds__(kBlock) void k_ms_pull_chunks(GraphArgs g, int lc,
                                                           const uint32_t* __restrict__ list,
                                                           const unsigned long long* marked,
                                                           uint64_t all,
                                                           const uint64_t* __restrict__ visited,
                                                           const uint64_t* __restrict__ cur,
                                                           uint64_t* __restrict__ nxt,
                                                           uint64_t* __restrict__ fbits,
                                                           uint32_t* __restrict__ fsum) {
    const uint64_t K = *marked >> kDegBits;
    const uint64_t slots = chunk_slots(K, lc);
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t s0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * R;
         s0 < slots; s0 += nwaves * R)
        ms_pull_slots<R>(g, s0, slots, lc, list, K, all, visited, cur, nxt, fbits, fsum);
}

__global__ __launch_bounds__(kCompactWaves * 64) void k_ms_finalize(uint64_t* bits, uint64_t words,
                                                        uint32_t n, const uint32_t* row_off,
                                                        uint32_t* list, uint32_t* degpre,
                                                        Ctl* ctl, uint64_t* fcur,
                                                        uint64_t* visited, uint64_t* retire,
                                                        const uint64_t* nxt, uint32_t* lev,
                                                        uint32_t K, uint32_t level, uint32_t* fsum,
                                                        uint32_t* csum) {
    ms_finalize_block<kCompactWaves>(blockIdx.x, bits, words, n, row_off, list, degpre, ctl, fcur,
                                     visited, retire, nxt, lev, K, level, fsum, csum);
}

// Sources of a multi-source run: bit s of nxt[src[s]], and the vertex bit.
__global__ void k_ms_seed(const uint32_t* __restrict__ srcs, uint32_t K, uint64_t* nxt,
                          uint64_t* fbits, uint32_t* fsum) {
    const uint32_t s = threadIdx.x;
    if (blockIdx.x == 0 && s < K) {
        atomicOr(reinterpret_cast<unsigned long long*>(nxt + srcs[s]), 1ull << s);
        set_bit_sum(fbits, fsum, srcs[s]);
    }
}

// Roots of a multi-root BFS: level 0 and the vertex bit.
__global__ void k_roots_seed(const uint32_t* __restrict__ roots, uint32_t count,
                             uint32_t* __restrict__ level, uint64_t* fbits, uint32_t* fsum) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        level[roots[i]] = 0;
        set_bit_sum(fbits, fsum, roots[i]);
    }
}

// Caller layout of multi-source levels: out[s*n + v] = lev[perm[v]*K + s], a
// transpose staged through LDS in tiles of 64 vertices x K sources: a wave
// reads one vertex's row of K levels (one coalesced load), and writes one
// source's 64 consecutive vertices (one coalesced store).
constexpr int kOutTile = 64;
__global__ __launch_bounds__(kBlock) void k_ms_output(uint32_t n, uint32_t K,
                                                      const uint32_t* __restrict__ perm,
                                                      const uint32_t* __restrict__ lev,
                                                      uint32_t* __restrict__ out) {
    __shared__ uint32_t tile[kOutTile][kOutTile + 1];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    for (uint64_t v0 = (uint64_t)blockIdx.x * kOutTile; v0 < n; v0 += (uint64_t)gridDim.x * kOutTile) {
        for (int r = wave; r < kOutTile; r += kWavesPerBlock) {
            const uint64_t v = v0 + r;
            if (v < n && (uint32_t)lane < K)
                tile[r][lane] = lev[(uint64_t)(perm ? perm[v] : (uint32_t)v) * K + lane];
        }
        __syncthreads();
        for (uint32_t s = wave; s < K; s += kWavesPerBlock) {
            const uint64_t v = v0 + lane;
            if (v < n) out[(uint64_t)s * n + v] = tile[lane][s];
        }
        __syncthreads();
    }
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t count, uint64_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_fill_u32b(uint32_t* __restrict__ p, uint64_t count, uint32_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ------------------------------------------------------- persistent kernel
//
// One launch runs every iteration: the blocks stride over each phase's work,
// separated by grid-wide barriers. Every block takes the fullness-gate
// decision itself from the same device counters, so the decision needs no
// barrier of its own. The grid is sized from the occupancy API so that every
// block is resident; each barrier wait is additionally bounded by a
// wall-clock deadline, after which the kernel records an error and every
// block exits.

// One block per CU holding all the waves the kernel's registers allow (2 per
// SIMD with the multi-source masks, 3 single-source): the same resident waves
// as several smaller blocks, but fewer blocks pay the per-block release at
// every barrier.
constexpr int kPersistWavesMs = 8;
constexpr int kPersistWavesBfs = 12;

__device__ __forceinline__ unsigned ld_rlx(unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld_counter(unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_counter(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two-level barrier: a block arrives on its group's counter (block b is in
// group b mod G), the last block of a group arrives on the top counter, and
// the last group advances the generation that the other blocks wait on.
//
// One release and one acquire per block and barrier, no more: on this part an
// agent-scope release writes back the XCD's L2 and an acquire invalidates it,
// so the wait polls with relaxed loads (an acquire load per poll would
// invalidate the L2 under the blocks still at work). The generation read
// cannot be stale (coherence of one location: this thread has seen the
// current value, and it cannot advance before this block arrives), and the
// release fence keeps it ahead of the arrival.
__device__ bool grid_sync(PersistState* ps, uint64_t timeout_ticks) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned gen = ld_rlx(&ps->bar_gen);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned nb = gridDim.x;
        const unsigned groups = nb < (unsigned)kBarGroups ? nb : (unsigned)kBarGroups;
        const unsigned grp = blockIdx.x % groups;
        const unsigned members = (nb - grp + groups - 1) / groups;  // blocks b < nb with b % groups == grp
        bool released = false;
        if (atomicAdd(&ps->bar_grp[grp][0], 1u) == members - 1) {
            atomicExch(&ps->bar_grp[grp][0], 0u);
            __threadfence();
            if (atomicAdd(&ps->bar_top[0], 1u) == groups - 1) {
                atomicExch(&ps->bar_top[0], 0u);
                __threadfence();
                atomicAdd(&ps->bar_gen, 1u);
                released = true;
            }
        }
        if (!released) {
            const uint64_t deadline = wall_clock64() + timeout_ticks;
            while (ld_rlx(&ps->bar_gen) == gen) {
                if (ld_rlx(&ps->error)) { ok = 0; break; }
                if (wall_clock64() > deadline) {
                    atomicExch(&ps->error, 1u);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (ld_rlx(&ps->error)) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

template <bool MS, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_bfs_persistent(PersistParams P) {
    const GraphArgs g = P.g;
    const uint64_t fwords = ((uint64_t)P.n + 63) / 64;
    const uint64_t fblocks = (fwords + kCompactWords * WAVES - 1) / (kCompactWords * WAVES);
    const uint64_t gwave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    PersistState* ps = P.ps;
    uint64_t* ma = P.masks[0];
    uint64_t* mb = P.masks[1];
    __shared__ unsigned long long s_a, s_b;

    // the seeds were written as the output of "iteration -1": list them
    for (uint64_t vb = blockIdx.x; vb < fblocks; vb += gridDim.x) {
        if (MS) ms_finalize_block<WAVES>(vb, P.fbits, fwords, P.n, P.row_off, P.flist[0], P.degpre[0],
                                  &ps->cnt[0].c, P.fcur, P.visited, mb, ma, P.lev, P.K, 0u);
        else bfs_finalize_block<WAVES>(vb, P.fbits, fwords, P.n, P.row_off, P.flist[0], P.degpre[0],
                                &ps->cnt[0].c, P.fcur);
    }
    if (!grid_sync(ps, P.timeout_ticks)) return;

    unsigned prev_mode = 0;
    for (uint32_t k = 0;; ++k) {
        const int cur = k & 1;
        Ctl* C = &ps->cnt[cur].c;       // counters of F_k (and this iteration's chunk count)
        Ctl* N = &ps->cnt[cur ^ 1].c;   // counters being built for F_{k+1}
        if (threadIdx.x == 0) {
            s_a = ld_counter(&C->ftotal);
            s_b = ld_counter(&C->fnext);
        }
        __syncthreads();
        const unsigned long long fcount = s_a;
        const unsigned long long flisted = s_b >> kDegBits;
        const unsigned long long active = s_b & kDegMask;
        const bool done = fcount == 0 || k >= P.max_iters;
        const unsigned mode = done ? 0u
                            : P.gate == WEDGE_GATE_ALWAYS_WEDGE ? 1u
                            : P.gate == WEDGE_GATE_ALWAYS_FULL ? 0u
                            : (active < P.thr ? 1u : 0u);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            // N was last used by iteration k-1, which every block has finished
            // (its reads of N came before the barriers that closed k-1): close
            // k-1's record, then clear N for this iteration's commit, which
            // starts only after at least one more barrier
            if (k > 0 && k - 1 < P.trace_cap && prev_mode)
                P.trace[k - 1].marked_chunks = ld_counter(&N->marked) >> kDegBits;
            if (!done && k < P.trace_cap) {
                wedge_iter_record r;
                r.iter = k;
                r.mode = mode;
                r.chunk_edges = mode ? (1u << P.lc) : 0u;
                r.reserved = 0;
                r.frontier = fcount;
                r.active_edges = active;
                r.marked_chunks = 0;
                r.ms = 0.f;
                r.reserved2 = 0.f;
                P.trace[k] = r;
            }
            if (fcount != 0 && k >= P.max_iters) ps->not_converged = 1;
            ps->iters = k;
            st_counter(&N->fnext, 0ull);
            st_counter(&N->ftotal, 0ull);
            st_counter(&N->marked, 0ull);
        }
        prev_mode = mode;
        if (done) break;
        uint64_t* mcur = cur ? mb : ma;   // masks of F_k (multi-source)
        uint64_t* mnxt = cur ? ma : mb;   // masks being built for F_{k+1}
        if (mode) {
            const uint64_t twaves = (active + 64ull * kTranslateEpt - 1) / (64ull * kTranslateEpt);
            for (uint64_t w = gwave; w < twaves; w += nwaves)
                translate_wave<kTranslateEpt>(w, P.flist[cur], P.degpre[cur], (uint32_t)flisted,
                                              (uint32_t)active, P.row_off, P.pos, P.lc,
                                              reinterpret_cast<uint32_t*>(P.wbits), nullptr);
            if (!grid_sync(ps, P.timeout_ticks)) return;
            const uint64_t cblocks = (P.wwords + kCompactWords * WAVES - 1) / (kCompactWords * WAVES);
            for (uint64_t vb = blockIdx.x; vb < cblocks; vb += gridDim.x)
                bitmap_compact_block<false, false, false, kCompactWords, WAVES>(
                    vb, P.wbits, P.wwords, 0xFFFFFFFFu, nullptr, P.chunks, nullptr, &C->marked,
                    nullptr, nullptr, nullptr, nullptr);
            if (!grid_sync(ps, P.timeout_ticks)) return;
            if (threadIdx.x == 0) s_a = ld_counter(&C->marked) >> kDegBits;
            __syncthreads();
            const uint64_t K = s_a;
            const uint64_t slots = chunk_slots(K, P.lc);
            for (uint64_t s0 = gwave * kPullRows; s0 < slots; s0 += nwaves * kPullRows) {
                if (MS) {
                    ms_pull_slots<kPullRows>(g, s0, slots, P.lc, P.chunks, K, P.all, P.visited, mcur,
                                             mnxt, P.fbits, nullptr);
                } else {
                    const int lane = lane_id();
                    uint32_t p[kPullRows];
                    bool valid[kPullRows];
                    chunk_slot_rows_any<kPullRows>(s0, slots, lane, P.lc, P.chunks, K, g.m, p, valid);
                    pull_lanes<kBfs, kPullRows>(g, p, valid, k, P.level, nullptr, P.fcur, P.fbits, nullptr);
                }
            }
        } else {
            for (uint64_t r0 = gwave * kPullRows; r0 < g.rows; r0 += nwaves * kPullRows) {
                if (MS) {
                    ms_pull_rows<kPullRows>(g, r0, P.all, P.visited, mcur, mnxt, P.fbits, nullptr);
                } else {
                    const int lane = lane_id();
                    uint32_t p[kPullRows];
                    bool valid[kPullRows];
#pragma unroll
                    for (int i = 0; i < kPullRows; ++i) {
                        const uint64_t pp = (r0 + i) * 64 + lane;
                        valid[i] = pp < g.m;
                        p[i] = (uint32_t)pp;
                    }
                    pull_lanes<kBfs, kPullRows>(g, p, valid, k, P.level, nullptr, P.fcur, P.fbits, nullptr);
                }
            }
        }
        if (!grid_sync(ps, P.timeout_ticks)) return;
        for (uint64_t vb = blockIdx.x; vb < fblocks; vb += gridDim.x) {
            if (MS) ms_finalize_block<WAVES>(vb, P.fbits, fwords, P.n, P.row_off, P.flist[cur ^ 1],
                                      P.degpre[cur ^ 1], N, P.fcur, P.visited, mcur, mnxt, P.lev,
                                      P.K, k + 1);
            else bfs_finalize_block<WAVES>(vb, P.fbits, fwords, P.n, P.row_off, P.flist[cur ^ 1],
                                    P.degpre[cur ^ 1], N, P.fcur);
        }
        if (!grid_sync(ps, P.timeout_ticks)) return;
    }
}

uint32_t grid_for(uint64_t threads, uint32_t cap) {
    uint64_t b = (threads + kBlock - 1) / kBlock;
    if (b == 0) b = 1;
    return (uint32_t)(b < cap ? b : cap);
}

}  // namespace

// ------------------------------------------------------------- launchers

template <int R>
void ms_pull_full_rows(const DevGraph& g, uint64_t all, const uint64_t* visited, const uint64_t* cur,
                       uint64_t* nxt, uint64_t* fbits, uint32_t* fsum, hipStream_t s) {
    const uint64_t waves = (g.rows + R - 1) / R;
    const uint32_t blocks = (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    k_ms_pull_full<R><<<blocks, kBlock, 0, s>>>(args_of(g), all, visited, cur, nxt, fbits, fsum);
}

hipError_t launch_ms_pull_full(const DevGraph& g, uint64_t all, const uint64_t* visited,
                               const uint64_t* cur, uint64_t* nxt, uint64_t* fbits, uint32_t* fsum,
                               hipStream_t s, int rows) {
    if (!g.rows) return hipSuccess;
    switch (rows) {
        case 4: ms_pull_full_rows<4>(g, all, visited, cur, nxt, fbits, fsum, s); break;
        case kPullRows: ms_pull_full_rows<kPullRows>(g, all, visited, cur, nxt, fbits, fsum, s); break;
        case 16: ms_pull_full_rows<16>(g, all, visited, cur, nxt, fbits, fsum, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int R>
void ms_pull_chunks_rows(const DevGraph& g, int lc, const uint32_t* list, const Ctl* ctl,
                         uint64_t max_chunks, uint64_t all, const uint64_t* visited,
                         const uint64_t* cur, uint64_t* nxt, uint64_t* fbits, uint32_t* fsum,
                         hipStream_t s) {
    uint64_t waves = (chunk_slots_count(max_chunks, lc) + R - 1) / R;
    if (waves > 256ull * 32) waves = 256ull * 32;
    const uint32_t blocks = (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    k_ms_pull_chunks<R><<<blocks, kBlock, 0, s>>>(args_of(g), lc, list, &ctl->marked, all, visited,
                                                  cur, nxt, fbits, fsum);
}

hipError_t launch_ms_pull_chunks(const DevGraph& g, int lc, const uint32_t* list, const Ctl* ctl,
                                 uint64_t max_chunks, uint64_t all, const uint64_t* visited,
                                 const uint64_t* cur, uint64_t* nxt, uint64_t* fbits, uint32_t* fsum,
                                 hipStream_t s, int rows) {
    if (!max_chunks) return hipSuccess;
    switch (rows) {
        case 4: ms_pull_chunks_rows<4>(g, lc, list, ctl, max_chunks, all, visited, cur, nxt, fbits, fsum, s); break;
        case kPullRows: ms_pull_chunks_rows<kPullRows>(g, lc, list, ctl, max_chunks, all, visited, cur, nxt, fbits, fsum, s); break;
        case 16: ms_pull_chunks_rows<16>(g, lc, list, ctl, max_chunks, all, visited, cur, nxt, fbits, fsum, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ms_finalize(uint64_t* fbits, uint32_t n, const uint32_t* row_off,
                              uint32_t* flist, uint32_t* degpre, Ctl* ctl, uint64_t* fcur,
                              uint64_t* visited, uint64_t* retire, const uint64_t* nxt,
                              uint32_t* lev, uint32_t K, uint32_t level, uint32_t* fsum,
                              uint32_t* csum, hipStream_t s) {
    const uint64_t words = ((uint64_t)n + 63) / 64;
    if (!words) return hipSuccess;
    const uint64_t waves = (words + kCompactWords - 1) / kCompactWords;
    const uint32_t blocks = (uint32_t)((waves + kCompactWaves - 1) / kCompactWaves);
    k_ms_finalize<<<blocks, kCompactWaves * 64, 0, s>>>(fbits, words, n, row_off, flist, degpre, ctl,
                                                        fcur, visited, retire, nxt, lev, K, level,
                                                        fsum, csum);
    return hipGetLastError();
}

hipError_t launch_ms_seed(const uint32_t* srcs, uint32_t K, uint64_t* nxt, uint64_t* fbits,
                          uint32_t* fsum, hipStream_t s) {
    k_ms_seed<<<1, 64, 0, s>>>(srcs, K, nxt, fbits, fsum);
    return hipGetLastError();
}

hipError_t launch_roots_seed(const uint32_t* roots, uint32_t count, uint32_t* level,
                             uint64_t* fbits, uint32_t* fsum, hipStream_t s) {
    if (!count) return hipSuccess;
    k_roots_seed<<<grid_for(count, 1024), kBlock, 0, s>>>(roots, count, level, fbits, fsum);
    return hipGetLastError();
}

hipError_t launch_ms_output(uint32_t n, uint32_t K, const uint32_t* perm, const uint32_t* lev,
                            uint32_t* out, hipStream_t s) {
    if (!n) return hipSuccess;
    if (K > kOutTile) return hipErrorInvalidValue;
    const uint64_t tiles = ((uint64_t)n + kOutTile - 1) / kOutTile;
    k_ms_output<<<(uint32_t)std::min<uint64_t>(tiles, 65536), kBlock, 0, s>>>(n, K, perm, lev, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t s) {
    if (!count) return hipSuccess;
    k_fill_u64<<<grid_for(count, 8192), kBlock, 0, s>>>(p, count, value);
    return hipGetLastError();
}

hipError_t launch_fill_u32_kernel(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s) {
    if (!count) return hipSuccess;
    k_fill_u32b<<<grid_for(count, 8192), kBlock, 0, s>>>(p, count, value);
    return hipGetLastError();
}

hipError_t persistent_max_blocks(bool ms, int* blocks_per_cu) {
    return ms ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_bfs_persistent<true, kPersistWavesMs>,
                                                             kPersistWavesMs * 64, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_bfs_persistent<false, kPersistWavesBfs>,
                                                             kPersistWavesBfs * 64, 0);
}

hipError_t launch_bfs_persistent(bool ms, const PersistParams& P, uint32_t blocks, hipStream_t s) {
    if (ms) k_bfs_persistent<true, kPersistWavesMs><<<blocks, kPersistWavesMs * 64, 0, s>>>(P);
    else k_bfs_persistent<false, kPersistWavesBfs><<<blocks, kPersistWavesBfs * 64, 0, s>>>(P);
    return hipGetLastError();
}

WEDGE_DEBUG_ACCESSOR(debug_take_batch)

}  // namespace wedge
