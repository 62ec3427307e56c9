// Learned gate: a small FP32 MLP (8 -> 32 -> 32 -> 4, ReLU) that predicts the
// log-time of the next iteration in each mode {full pull, Wedge Frontier at 16,
// 32, 64 edges per bit} relative to the full pull; a model is an ensemble of
// such MLPs (independently initialised and trained) whose predictions are
// averaged, and the gate picks the smallest mean prediction. Inference
// runs on one wave between iterations from the device counters; training is a
// per-sample forward/backward with LDS-reduced gradients and an Adam update.
// The paper's threshold rule (Frontier Transformation, Frontier Fullness
// Threshold) is the fallback whenever a feature leaves the training envelope.
#include <math.h>

#include "device_common.h"

namespace wedge {
namespace {

using namespace dev;

// parameter layout (row-major, out x in)
constexpr int kW1 = 0;
constexpr int kB1 = kW1 + kMlpHidden * kMlpIn;
constexpr int kW2 = kB1 + kMlpHidden;
constexpr int kB2 = kW2 + kMlpHidden * kMlpHidden;
constexpr int kW3 = kB2 + kMlpHidden;
constexpr int kB3 = kW3 + kMlpOut * kMlpHidden;
static_assert(kB3 + kMlpOut == kMlpParams, "parameter count");

// Forward pass of one sample held by one thread; keeps activations for backward.
__device__ __forceinline__ void mlp_forward(const float* __restrict__ P, const float (&x)[kMlpIn],
                                            float (&h1)[kMlpHidden], float (&h2)[kMlpHidden],
                                            float (&y)[kMlpOut]) {
#pragma unroll 4
    for (int j = 0; j < kMlpHidden; ++j) {
        float a = P[kB1 + j];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) a += P[kW1 + j * kMlpIn + i] * x[i];
        h1[j] = a > 0.f ? a : 0.f;
    }
#pragma unroll 4
    for (int j = 0; j < kMlpHidden; ++j) {
        float a = P[kB2 + j];
        for (int i = 0; i < kMlpHidden; ++i) a += P[kW2 + j * kMlpHidden + i] * h1[i];
        h2[j] = a > 0.f ? a : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kMlpOut; ++j) {
        float a = P[kB3 + j];
        for (int i = 0; i < kMlpHidden; ++i) a += P[kW3 + j * kMlpHidden + i] * h2[i];
        y[j] = a;
    }
}

// Features of the frontier the next iteration will consume (see mlp_features).
__device__ __forceinline__ void make_features(float (&x)[kMlpIn], double fcount, double active,
                                              double n, double m, double k, double prev_us,
                                              double prev_mode, double app) {
    x[0] = (float)(fcount / n);
    x[1] = (float)(active / m);
    x[2] = (float)(1.0 - exp(-active / ceil(m / 16.0)));
    x[3] = (float)(app / 3.0);
    x[4] = (float)(log2(m) / 32.0);
    x[5] = (float)(fmin(k, 255.0) / 64.0);
    x[6] = (float)(log1p(prev_us) / 16.0);
    x[7] = (float)(prev_mode / 3.0);
}

// Batched forward for evaluation: Y[b] = mean over the ensemble's members of
// MLP_e(X[b]).
__global__ __launch_bounds__(kBlock) void k_mlp_forward(const float* __restrict__ P, uint32_t members,
                                                        const float* __restrict__ X,
                                                        float* __restrict__ Y, uint32_t count) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    float x[kMlpIn], h1[kMlpHidden], h2[kMlpHidden], y[kMlpOut], acc[kMlpOut];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) x[i] = X[(uint64_t)b * kMlpIn + i];
#pragma unroll
    for (int j = 0; j < kMlpOut; ++j) acc[j] = 0.f;
    for (uint32_t e = 0; e < members; ++e) {
        mlp_forward(P + (size_t)e * kMlpParams, x, h1, h2, y);
#pragma unroll
        for (int j = 0; j < kMlpOut; ++j) acc[j] += y[j];
    }
#pragma unroll
    for (int j = 0; j < kMlpOut; ++j) Y[(uint64_t)b * kMlpOut + j] = acc[j] / (float)members;
}

// Gradient of the mean squared error over the sample's target outputs
// (target components with a zero mask are ignored), summed over the batch into
// G. Each block sums its samples in LDS and adds its total to G once per
// parameter.
__global__ __launch_bounds__(kBlock) void k_mlp_grad(const float* __restrict__ P,
                                                     const float* __restrict__ X,
                                                     const float* __restrict__ T,
                                                     const float* __restrict__ Mk, uint32_t count,
                                                     float scale, float* __restrict__ G,
                                                     float* __restrict__ loss) {
    __shared__ float sg[kMlpParams];
    __shared__ float sl;
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) sg[i] = 0.f;
    if (threadIdx.x == 0) sl = 0.f;
    __syncthreads();
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < count) {
        float x[kMlpIn], h1[kMlpHidden], h2[kMlpHidden], y[kMlpOut];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) x[i] = X[(uint64_t)b * kMlpIn + i];
        mlp_forward(P, x, h1, h2, y);
        float dy[kMlpOut];
        float l = 0.f;
#pragma unroll
        for (int j = 0; j < kMlpOut; ++j) {
            const float mk = Mk[(uint64_t)b * kMlpOut + j];
            const float e = (y[j] - T[(uint64_t)b * kMlpOut + j]) * mk;
            l += e * e;
            dy[j] = 2.f * e * scale;
        }
        atomicAdd(&sl, l * scale);
        // layer 3
        float dh2[kMlpHidden];
        for (int i = 0; i < kMlpHidden; ++i) dh2[i] = 0.f;
#pragma unroll
        for (int j = 0; j < kMlpOut; ++j) {
            atomicAdd(&sg[kB3 + j], dy[j]);
            for (int i = 0; i < kMlpHidden; ++i) {
                atomicAdd(&sg[kW3 + j * kMlpHidden + i], dy[j] * h2[i]);
                dh2[i] += dy[j] * P[kW3 + j * kMlpHidden + i];
            }
        }
        // layer 2
        float dh1[kMlpHidden];
        for (int i = 0; i < kMlpHidden; ++i) dh1[i] = 0.f;
        for (int j = 0; j < kMlpHidden; ++j) {
            const float d = h2[j] > 0.f ? dh2[j] : 0.f;
            if (d == 0.f) continue;
            atomicAdd(&sg[kB2 + j], d);
            for (int i = 0; i < kMlpHidden; ++i) {
                atomicAdd(&sg[kW2 + j * kMlpHidden + i], d * h1[i]);
                dh1[i] += d * P[kW2 + j * kMlpHidden + i];
            }
        }
        // layer 1
        for (int j = 0; j < kMlpHidden; ++j) {
            const float d = h1[j] > 0.f ? dh1[j] : 0.f;
            if (d == 0.f) continue;
            atomicAdd(&sg[kB1 + j], d);
#pragma unroll
            for (int i = 0; i < kMlpIn; ++i) atomicAdd(&sg[kW1 + j * kMlpIn + i], d * x[i]);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x)
        if (sg[i] != 0.f) atomicAdd(&G[i], sg[i]);
    if (threadIdx.x == 0 && loss) atomicAdd(loss, sl);
}

// Adam (Kingma & Ba 2015) on every parameter; clears the gradient.
__global__ void k_adam(float* __restrict__ P, float* __restrict__ G, float* __restrict__ M1,
                       float* __restrict__ M2, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    const float g = G[i];
    const float m = b1 * M1[i] + (1.f - b1) * g;
    const float v = b2 * M2[i] + (1.f - b2) * g * g;
    M1[i] = m;
    M2[i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    G[i] = 0.f;
}

// Decision for the next iteration from the device counters. One wave:
// lanes 0..31 compute the hidden units of each layer, lane 0 the outputs and
// the argmin (ties go to the lowest mode index). Features outside the
// training envelope, or no model, fall back to the threshold rule.
// The decision is left in ctl->gate for the host's per-iteration read-back.
__device__ __forceinline__ uint32_t mode_of_lc(uint32_t lc) {
    return lc <= 4 ? 1u : lc == 5 ? 2u : 3u;
}

// Start of an iteration: clear the iteration counters and stamp the time (the
// previous-iteration-time feature is the device time from this stamp to the
// next decision).
__global__ void k_gate_stamp(Ctl* ctl) {
    if (threadIdx.x == 0) {
        ctl->fnext = 0;
        ctl->marked = 0;
        ctl->ftotal = 0;
        ctl->gate.stamp = wall_clock64();
    }
}

// One wave per ensemble member (block of 64 x members threads), so the
// members' three dependent layers run side by side rather than one after
// another; the outputs are summed in member order, as before.
__global__ __launch_bounds__(64 * kMlpMaxMembers) void k_mlp_infer(
    const float* __restrict__ P, uint32_t members, const float* __restrict__ env_lo,
    const float* __restrict__ env_hi, float margin, Ctl* ctl, double n, double m, uint64_t thr,
    uint32_t fallback_lc, double ticks_per_us, uint32_t app) {
    GateState* gs = &ctl->gate;
    __shared__ float h1[kMlpMaxMembers][kMlpHidden], h2[kMlpMaxMembers][kMlpHidden];
    __shared__ float out[kMlpMaxMembers][kMlpOut];
    __shared__ float xs[kMlpIn];
    __shared__ int s_in;
    const int lane = threadIdx.x & 63;
    const uint32_t e = threadIdx.x >> 6;
    const uint64_t now = wall_clock64();
    const double fcount = (double)ctl->ftotal;
    const unsigned long long active = ctl->fnext & kDegMask;
    if (threadIdx.x == 0) {
        const double prev_us = gs->stamp ? (double)(now - gs->stamp) / ticks_per_us : 0.0;
        float x[kMlpIn];
        make_features(x, fcount, (double)active, n, m, (double)gs->k, prev_us, (double)gs->prev_mode,
                      (double)app);
        int in = P != nullptr;
        for (int i = 0; i < kMlpIn; ++i) {
            xs[i] = x[i];
            if (P && (x[i] < env_lo[i] || x[i] > env_hi[i])) in = 0;
        }
        s_in = in;
    }
    __syncthreads();
    const bool run = s_in && e < members;
    const float* Q = P + (size_t)(run ? e : 0) * kMlpParams;
    if (run && lane < kMlpHidden) {
        float a = Q[kB1 + lane];
        for (int i = 0; i < kMlpIn; ++i) a += Q[kW1 + lane * kMlpIn + i] * xs[i];
        h1[e][lane] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (run && lane < kMlpHidden) {
        float a = Q[kB2 + lane];
        for (int i = 0; i < kMlpHidden; ++i) a += Q[kW2 + lane * kMlpHidden + i] * h1[e][i];
        h2[e][lane] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (run && lane < kMlpOut) {
        float a = Q[kB3 + lane];
        for (int i = 0; i < kMlpHidden; ++i) a += Q[kW3 + lane * kMlpHidden + i] * h2[e][i];
        out[e][lane] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the ensemble's summed outputs (argmin of the sum = argmin of the mean)
        float acc[kMlpOut] = {0.f, 0.f, 0.f, 0.f};
        if (s_in)
            for (uint32_t k = 0; k < members; ++k)
                for (int j = 0; j < kMlpOut; ++j) acc[j] += out[k][j];
        uint32_t mode = 0, lc = fallback_lc;
        if (s_in) {
            // the model's choice (argmin, ties to the lower index) replaces the
            // threshold rule's only when its predicted mean log-time is lower
            // than that of the rule's choice by more than the margin
            uint32_t jb = 0;
            for (int j = 1; j < kMlpOut; ++j)
                if (acc[j] < acc[jb]) jb = j;
            const bool thr_wedge = active < thr;
            const uint32_t jt = thr_wedge ? mode_of_lc(fallback_lc) : 0u;
            if (jb != jt && acc[jt] - acc[jb] > margin * (float)members) {
                mode = jb;
                lc = mode ? 3 + mode : fallback_lc;  // modes 1, 2, 3 = 16, 32, 64 edges per bit
            } else {
                mode = jt;
                lc = fallback_lc;
            }
            gs->learned++;
        } else {
            mode = active < thr ? 1u : 0u;         // the threshold rule
            gs->fallback++;
        }
        gs->mode = mode ? 1u : 0u;
        gs->lc = lc;
        gs->prev_mode = mode ? (s_in ? mode : mode_of_lc(lc)) : 0u;
        gs->k++;
    }
}

}  // namespace

hipError_t launch_mlp_forward(const float* P, uint32_t members, const float* X, float* Y,
                              uint32_t count, hipStream_t s) {
    if (!count) return hipSuccess;
    k_mlp_forward<<<(count + kBlock - 1) / kBlock, kBlock, 0, s>>>(P, members, X, Y, count);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, const float* Mk,
                           uint32_t count, float scale, float* G, float* loss, hipStream_t s) {
    if (!count) return hipSuccess;
    k_mlp_grad<<<(count + kBlock - 1) / kBlock, kBlock, 0, s>>>(P, X, T, Mk, count, scale, G, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* P, float* G, float* M1, float* M2, float lr, float b1, float b2,
                       float eps, uint32_t step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    k_adam<<<(kMlpParams + kBlock - 1) / kBlock, kBlock, 0, s>>>(P, G, M1, M2, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* P, uint32_t members, const float* lo, const float* hi,
                            float margin, Ctl* ctl, double n, double m, uint64_t thr,
                            uint32_t fallback_lc, double ticks_per_us, uint32_t app, hipStream_t s) {
    const uint32_t waves = P ? (members < 1 ? 1u : members > kMlpMaxMembers ? kMlpMaxMembers : members) : 1u;
    k_mlp_infer<<<1, 64 * waves, 0, s>>>(P, waves, lo, hi, margin, ctl, n, m, thr, fallback_lc, ticks_per_us, app);
    return hipGetLastError();
}

hipError_t launch_gate_stamp(Ctl* ctl, hipStream_t s) {
    k_gate_stamp<<<1, 64, 0, s>>>(ctl);
    return hipGetLastError();
}

}  // namespace wedge
