// Push engine on gfx950: the baseline the paper's method replaces.
//
// A push iteration walks the out-edges of the frontier's vertices and sends
// each source's value to the destination (Background, Push vs. Pull: the
// engine aligned with the source-oriented frontier). Destinations are updated
// with atomics, because many sources may send to one destination in the same
// iteration. With it the library can run the hybrid engines the paper
// compares against (Background, Hybrid Graph Processing: push when the
// frontier's out-edges are few, a pull over the whole graph otherwise) on the
// same GPU, graphs and applications as the Wedge Frontier.
//
// Iteration semantics are those of the pull engine (synchronous: sources send
// the value committed at the end of the previous iteration, and a vertex joins
// the next frontier exactly when its value drops), so every engine produces
// the same values and the same frontier in every iteration.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace wedge {
namespace {

using namespace dev;

constexpr int kPushEpt = 4;  // frontier out-edges per lane (rows of 64 per wave)

// Out-edge arrays of the push engine, in CSR order: the destination of out-edge
// q is the vertex that owns in-edge position pos[q] (read off the row layout),
// and its weight is the weight stored at that position.
__global__ __launch_bounds__(kBlock) void k_out_edges(GraphArgs g, const uint32_t* __restrict__ pos,
                                                      uint32_t* __restrict__ out_dst,
                                                      uint32_t* __restrict__ out_w) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < g.m; q += stride) {
        const uint32_t p = pos[q];
        const uint64_t mk = g.rowmask[p >> 6];
        const uint32_t sg = g.rowseg[p >> 6];
        out_dst[q] = g.nzdst[sg + (uint32_t)__popcll(mk & ~1ull & mask_le((int)(p & 63)))];
        if (out_w) out_w[q] = g.in_w[p];
    }
}

// One push iteration. Work is split by out-edges, as in the frontier
// transformation: lane j of wave w takes edge a = w*64*EPT + i*64 + j of the
// concatenated out-edge lists of the listed frontier (degpre is its exclusive
// out-degree prefix) and finds the edge's source by a shuffle search in a
// window of 64 list entries. Per edge:
//   BFS      : an unvisited destination gets level k+1;
//   CC, SSSP : candidate = committed value of the source (+ weight for SSSP);
//              when it is below the destination's current value, a min-atomic
//              lowers the destination (nothing waits for the atomic: a value
//              only falls within an iteration, so a candidate below any value
//              read proves the destination changes).
// A destination that changes gets its next-frontier bit.
template <int APP, int EPT>
__global__ __launch_bounds__(kBlock) void k_push(const uint32_t* __restrict__ flist,
                                                 const uint32_t* __restrict__ degpre,
                                                 uint32_t fcount, uint32_t active,
                                                 const uint32_t* __restrict__ row_off,
                                                 const uint32_t* __restrict__ out_dst,
                                                 const uint32_t* __restrict__ out_w, uint32_t iter,
                                                 uint32_t* __restrict__ val,
                                                 const uint32_t* __restrict__ val_prev,
                                                 uint64_t* __restrict__ fbits,
                                                 uint32_t* __restrict__ fsum) {
    const int lane = lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t base = wave * 64ull * EPT;
    if (base >= active) return;
    const uint64_t end = umin64(base + 64ull * EPT, active);
    uint32_t j0 = wave_last_le(degpre, 0, fcount - 1, base, lane);
    uint32_t q[EPT], x[EPT];
    bool valid[EPT];
    // owners of the wave's edges, row by row (each row's window starts where
    // the previous row's last edge lies)
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const uint64_t row = base + (uint64_t)i * 64;
        const uint64_t a = row + lane;
        valid[i] = a < end;
        q[i] = 0;
        x[i] = 0;
        if (row >= end) continue;  // wave-uniform
        const uint32_t jw = j0 + lane;
        const bool in = jw < fcount;
        const uint32_t uw = in ? flist[jw] : 0u;
        const uint32_t dw = in ? degpre[jw] : 0xFFFFFFFFu;
        const uint32_t rw = row_off[uw];
        const uint32_t xw = APP == kBfs ? 0u : val_prev[uw];
        int t = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const int cand = t + step;
            const uint32_t d = __shfl(dw, cand & 63, 64);
            if (cand < 64 && d <= a) t = cand;
        }
        const uint32_t dt = __shfl(dw, t, 64);
        const uint32_t rt = __shfl(rw, t, 64);
        x[i] = __shfl(xw, t, 64);
        q[i] = valid[i] ? rt + (uint32_t)(a - dt) : 0u;
        // every listed vertex has an out-edge, so the window of 64 entries
        // from the owner of edge row + 63 (or the next one) covers the next row
        j0 += lane_bcast((uint32_t)t, 63);
        if (j0 + 1 < fcount && degpre[j0 + 1] <= row + 64) ++j0;
    }
    // every row's edge loads, then every row's destination value, then the updates
    uint32_t v[EPT], w[EPT], cur[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) v[i] = ld_stream(out_dst + q[i]);
#pragma unroll
    for (int i = 0; i < EPT; ++i) w[i] = APP == kSssp ? ld_stream(out_w + q[i]) : 0u;
#pragma unroll
    for (int i = 0; i < EPT; ++i) cur[i] = val[v[i]];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        if (!valid[i]) continue;
        if (APP == kBfs) {
            if (cur[i] == kInf) {
                val[v[i]] = iter + 1;
                set_bit_sum(fbits, fsum, v[i]);
            }
        } else {
            const uint32_t cand = (APP == kCc || x[i] == kInf) ? x[i] : x[i] + w[i];
            if (cand < cur[i]) {
                atomicMin(val + v[i], cand);
                set_bit_sum(fbits, fsum, v[i]);
            }
        }
    }
}

}  // namespace

hipError_t launch_out_edges(const DevGraph& g, const uint32_t* pos, uint32_t* out_dst, uint32_t* out_w,
                            hipStream_t s) {
    if (!g.m) return hipSuccess;
    uint64_t blocks = (g.m + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    k_out_edges<<<(uint32_t)blocks, kBlock, 0, s>>>(args_of(g), pos, out_dst, out_w);
    return hipGetLastError();
}

hipError_t launch_push(int app, const uint32_t* flist, const uint32_t* degpre, uint32_t fcount,
                       uint64_t active, const uint32_t* row_off, const uint32_t* out_dst,
                       const uint32_t* out_w, uint32_t iter, uint32_t* val, const uint32_t* val_prev,
                       uint64_t* fbits, uint32_t* fsum, hipStream_t s) {
    if (!fcount || !active) return hipSuccess;
    if (app == kSssp && !out_w) return hipErrorInvalidValue;
    if (app != kBfs && !val_prev) return hipErrorInvalidValue;
    const uint64_t waves = (active + 64ull * kPushEpt - 1) / (64ull * kPushEpt);
    const uint32_t blocks = (uint32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    const uint32_t a = (uint32_t)active;
    if (app == kBfs)
        k_push<kBfs, kPushEpt><<<blocks, kBlock, 0, s>>>(flist, degpre, fcount, a, row_off, out_dst,
                                                         out_w, iter, val, val_prev, fbits, fsum);
    else if (app == kCc)
        k_push<kCc, kPushEpt><<<blocks, kBlock, 0, s>>>(flist, degpre, fcount, a, row_off, out_dst,
                                                        out_w, iter, val, val_prev, fbits, fsum);
    else
        k_push<kSssp, kPushEpt><<<blocks, kBlock, 0, s>>>(flist, degpre, fcount, a, row_off, out_dst,
                                                          out_w, iter, val, val_prev, fbits, fsum);
    return hipGetLastError();
}

WEDGE_DEBUG_ACCESSOR(debug_take_push)

}  // namespace wedge
