// Learned-gate model on the host side: creation, file format, training and
// prediction (the arithmetic runs in the HIP kernels of mlp.hip).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "wedge_internal.h"

using namespace wedge;

namespace {

constexpr char kMagic[8] = {'W', 'E', 'D', 'G', 'E', 'M', 'L', 'P'};
constexpr uint32_t kVersion = 4;  // 4: + decision margin; 3: ensemble (member count); 2: one MLP

wedge_status err(wedge_status st, const std::string& m) { return set_error(st, m); }

#define HTRY(expr, what)                                                              \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) return err(WEDGE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(_e)); \
    } while (0)

uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 1469598103934665603ull) {
    for (size_t i = 0; i < n; ++i) { h ^= p[i]; h *= 1099511628211ull; }
    return h;
}

uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void free_device(wedge_model_s* m) {
    wedge::SetupLock lock;
    if (m->dev_params) (void)hipFree(m->dev_params);
    if (m->dev_lo) (void)hipFree(m->dev_lo);
    if (m->dev_hi) (void)hipFree(m->dev_hi);
    m->dev_params = m->dev_lo = m->dev_hi = nullptr;
    m->device = -1;
    m->dirty = true;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (!p) return;
        wedge::SetupLock lock;
        (void)hipFree(p);
    }
};

}  // namespace

namespace wedge {

void mlp_features(float* x, double fcount, double active, double n, double m, double k,
                  double prev_us, double prev_mode, double app) {
    x[0] = (float)(fcount / n);
    x[1] = (float)(active / m);
    x[2] = (float)(1.0 - std::exp(-active / std::ceil(m / 16.0)));
    x[3] = (float)(app / 3.0);
    x[4] = (float)(std::log2(m) / 32.0);
    x[5] = (float)(std::fmin(k, 255.0) / 64.0);
    x[6] = (float)(std::log1p(prev_us) / 16.0);
    x[7] = (float)(prev_mode / 3.0);
}

wedge_status model_to_device(wedge_model_s* m) {
    SetupLock lock;
    int dev = 0;
    HTRY(hipGetDevice(&dev), "hipGetDevice");
    if (m->dev_params && m->device != dev) free_device(m);
    const size_t np = (size_t)m->members * kMlpParams;
    // each buffer is allocated when missing, so a failed upload is completed
    // by the next one rather than leaving null buffers behind
    if (!m->dev_params || !m->dev_lo || !m->dev_hi) {
        m->dirty = true;
        if (!m->dev_params) {
            HTRY(hipMalloc((void**)&m->dev_params, np * sizeof(float)), "model parameters");
            m->device = dev;
        }
        if (!m->dev_lo) HTRY(hipMalloc((void**)&m->dev_lo, kMlpIn * sizeof(float)), "model envelope");
        if (!m->dev_hi) HTRY(hipMalloc((void**)&m->dev_hi, kMlpIn * sizeof(float)), "model envelope");
    }
    if (m->dirty) {
        HTRY(hipMemcpy(m->dev_params, m->params.data(), np * sizeof(float), hipMemcpyHostToDevice), "model upload");
        HTRY(hipMemcpy(m->dev_lo, m->lo.data(), kMlpIn * sizeof(float), hipMemcpyHostToDevice), "model upload");
        HTRY(hipMemcpy(m->dev_hi, m->hi.data(), kMlpIn * sizeof(float), hipMemcpyHostToDevice), "model upload");
        m->dirty = false;
    }
    return WEDGE_OK;
}

}  // namespace wedge

extern "C" {

wedge_status wedge_model_create_ensemble(uint64_t seed, uint32_t members, wedge_model_t* out) {
    if (!out) return err(WEDGE_ERR_INVALID_ARG, "out is null");
    if (members < 1 || members > kMlpMaxMembers) return err(WEDGE_ERR_INVALID_ARG, "members must be 1..8");
    try {
        auto* m = new wedge_model_s();
        m->members = members;
        m->params.assign((size_t)members * kMlpParams, 0.f);
        m->lo.assign(kMlpIn, -std::numeric_limits<float>::infinity());
        m->hi.assign(kMlpIn, std::numeric_limits<float>::infinity());
        // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases; the
        // members draw one after another from the same stream
        uint64_t s = seed;
        for (uint32_t e = 0; e < members; ++e) {
            float* P = m->params.data() + (size_t)e * kMlpParams;
            auto fill = [&](int off, int rows, int cols) {
                const double b = 1.0 / std::sqrt((double)cols);
                for (int i = 0; i < rows * cols; ++i) {
                    double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
                    P[off + i] = (float)((2.0 * u - 1.0) * b);
                }
            };
            const int w1 = 0, b1 = w1 + kMlpHidden * kMlpIn, w2 = b1 + kMlpHidden;
            const int b2 = w2 + kMlpHidden * kMlpHidden, w3 = b2 + kMlpHidden;
            fill(w1, kMlpHidden, kMlpIn);
            fill(w2, kMlpHidden, kMlpHidden);
            fill(w3, kMlpOut, kMlpHidden);
        }
        *out = m;
        return WEDGE_OK;
    } catch (const std::bad_alloc&) {
        return err(WEDGE_ERR_OOM, "host allocation failed");
    }
}

wedge_status wedge_model_create(uint64_t seed, wedge_model_t* out) {
    return wedge_model_create_ensemble(seed, 1, out);
}

wedge_status wedge_model_margin(wedge_model_t m, float* margin, int set) {
    if (!m || !margin) return err(WEDGE_ERR_INVALID_ARG, "null argument");
    if (set) {
        if (!std::isfinite(*margin) || *margin < 0.f) return err(WEDGE_ERR_INVALID_ARG, "margin must be finite and >= 0");
        m->margin = *margin;
    } else {
        *margin = m->margin;
    }
    return WEDGE_OK;
}

wedge_status wedge_model_members(wedge_model_t m, uint32_t* members) {
    if (!m || !members) return err(WEDGE_ERR_INVALID_ARG, "null argument");
    *members = m->members;
    return WEDGE_OK;
}

wedge_status wedge_model_free(wedge_model_t m) {
    if (!m) return WEDGE_OK;
    free_device(m);
    delete m;
    return WEDGE_OK;
}

wedge_status wedge_model_params(wedge_model_t m, float* params, uint32_t count, int set) {
    if (!m || !params) return err(WEDGE_ERR_INVALID_ARG, "null argument");
    const size_t np = (size_t)m->members * kMlpParams;
    if (count != np) return err(WEDGE_ERR_INVALID_ARG, "count must be 1476 x members");
    if (set) { std::memcpy(m->params.data(), params, np * sizeof(float)); m->dirty = true; }
    else std::memcpy(params, m->params.data(), np * sizeof(float));
    return WEDGE_OK;
}

wedge_status wedge_model_envelope(wedge_model_t m, float* lo, float* hi, int set) {
    if (!m || !lo || !hi) return err(WEDGE_ERR_INVALID_ARG, "null argument");
    if (set) {
        std::memcpy(m->lo.data(), lo, kMlpIn * sizeof(float));
        std::memcpy(m->hi.data(), hi, kMlpIn * sizeof(float));
        m->dirty = true;
    } else {
        std::memcpy(lo, m->lo.data(), kMlpIn * sizeof(float));
        std::memcpy(hi, m->hi.data(), kMlpIn * sizeof(float));
    }
    return WEDGE_OK;
}

wedge_status wedge_model_save(wedge_model_t m, const char* path) {
    if (!m || !path) return err(WEDGE_ERR_INVALID_ARG, "null argument");
    std::vector<unsigned char> buf;
    auto put = [&](const void* p, size_t n) {
        const unsigned char* c = static_cast<const unsigned char*>(p);
        buf.insert(buf.end(), c, c + n);
    };
    uint32_t margin_bits;
    std::memcpy(&margin_bits, &m->margin, 4);
    const uint32_t hdr[7] = {kVersion, (uint32_t)kMlpParams, (uint32_t)kMlpIn, (uint32_t)kMlpHidden,
                             (uint32_t)kMlpOut, m->members, margin_bits};
    put(kMagic, 8);
    put(hdr, sizeof hdr);
    put(m->lo.data(), kMlpIn * sizeof(float));
    put(m->hi.data(), kMlpIn * sizeof(float));
    put(m->params.data(), (size_t)m->members * kMlpParams * sizeof(float));
    const uint64_t sum = fnv1a(buf.data(), buf.size());
    put(&sum, sizeof sum);
    FILE* f = std::fopen(path, "wb");
    if (!f) return err(WEDGE_ERR_INVALID_ARG, std::string("cannot open ") + path);
    const size_t wr = std::fwrite(buf.data(), 1, buf.size(), f);
    std::fclose(f);
    if (wr != buf.size()) return err(WEDGE_ERR_INVALID_ARG, "short write");
    return WEDGE_OK;
}

wedge_status wedge_model_load(const char* path, wedge_model_t* out) {
    if (!path || !out) return err(WEDGE_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return err(WEDGE_ERR_MODEL, std::string("cannot open model file ") + path);
    std::vector<unsigned char> buf;
    unsigned char tmp[4096];
    size_t r;
    while ((r = std::fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + r);
    std::fclose(f);
    if (buf.size() < 8 + 5 * 4 || std::memcmp(buf.data(), kMagic, 8) != 0)
        return err(WEDGE_ERR_MODEL, "not a model file");
    uint32_t hdr[7] = {0, 0, 0, 0, 0, 1, 0};
    std::memcpy(hdr, buf.data() + 8, 5 * 4);
    // header words by version: 2 = five (one MLP), 3 = six (+ members),
    // 4 = seven (+ decision margin); older files load with margin 0
    const size_t hwords = hdr[0] == 2 ? 5 : hdr[0] == 3 ? 6 : 7;
    if ((hdr[0] == 3 || hdr[0] == 4) && buf.size() >= 8 + hwords * 4) std::memcpy(hdr, buf.data() + 8, hwords * 4);
    if (hdr[0] < 2 || hdr[0] > kVersion || hdr[1] != (uint32_t)kMlpParams ||
        hdr[2] != (uint32_t)kMlpIn || hdr[3] != (uint32_t)kMlpHidden || hdr[4] != (uint32_t)kMlpOut ||
        hdr[5] < 1 || hdr[5] > kMlpMaxMembers)
        return err(WEDGE_ERR_MODEL, "model version or shape mismatch");
    float margin = 0.f;
    std::memcpy(&margin, &hdr[6], 4);
    if (!std::isfinite(margin) || margin < 0.f) return err(WEDGE_ERR_MODEL, "model has an invalid margin");
    const size_t np = (size_t)hdr[5] * kMlpParams;
    const size_t want = 8 + hwords * 4 + 2 * kMlpIn * 4 + np * 4 + 8;
    if (buf.size() != want) return err(WEDGE_ERR_MODEL, "model file has the wrong size");
    uint64_t sum;
    std::memcpy(&sum, buf.data() + want - 8, 8);
    if (fnv1a(buf.data(), want - 8) != sum) return err(WEDGE_ERR_MODEL, "model checksum mismatch");
    auto* m = new wedge_model_s();
    const unsigned char* p = buf.data() + 8 + hwords * 4;
    m->members = hdr[5];
    m->margin = margin;
    m->lo.resize(kMlpIn);
    m->hi.resize(kMlpIn);
    m->params.resize(np);
    std::memcpy(m->lo.data(), p, kMlpIn * 4); p += kMlpIn * 4;
    std::memcpy(m->hi.data(), p, kMlpIn * 4); p += kMlpIn * 4;
    std::memcpy(m->params.data(), p, np * 4);
    for (float v : m->params)
        if (!std::isfinite(v)) { delete m; return err(WEDGE_ERR_MODEL, "model has non-finite parameters"); }
    *out = m;
    return WEDGE_OK;
}

wedge_status wedge_model_features(const wedge_trace_sample* s, uint32_t count, float* x) {
    if ((count && !s) || (count && !x)) return err(WEDGE_ERR_INVALID_ARG, "null argument");
    for (uint32_t i = 0; i < count; ++i)
        mlp_features(x + (size_t)i * kMlpIn, (double)s[i].frontier, (double)s[i].active,
                     (double)s[i].n, (double)s[i].m, (double)s[i].iter, (double)s[i].prev_us,
                     (double)s[i].prev_mode, (double)s[i].app);
    return WEDGE_OK;
}

wedge_status wedge_model_predict(wedge_model_t m, const float* x, uint32_t count, float* y,
                                 hipStream_t stream) {
    if (!m || (count && (!x || !y))) return err(WEDGE_ERR_INVALID_ARG, "null argument");
    if (!count) return WEDGE_OK;
    wedge_status st = model_to_device(m);
    if (st != WEDGE_OK) return st;
    DevBuf dx, dy;
    SetupLock alloc_lock;
    HTRY(hipMalloc(&dx.p, (size_t)count * kMlpIn * 4), "features");
    HTRY(hipMalloc(&dy.p, (size_t)count * kMlpOut * 4), "predictions");
    HTRY(hipMemcpyAsync(dx.p, x, (size_t)count * kMlpIn * 4, hipMemcpyHostToDevice, stream), "features");
    HTRY(launch_mlp_forward(m->dev_params, m->members, (const float*)dx.p, (float*)dy.p, count, stream),
         "forward");
    HTRY(hipMemcpyAsync(y, dy.p, (size_t)count * kMlpOut * 4, hipMemcpyDeviceToHost, stream), "predictions");
    HTRY(hipStreamSynchronize(stream), "prediction");
    return WEDGE_OK;
}

wedge_status wedge_model_grad(wedge_model_t m, const float* x, const float* t, const float* mask,
                              uint32_t count, float* grad, float* loss, hipStream_t stream) {
    if (!m || !x || !t || !mask || !grad || !count) return err(WEDGE_ERR_INVALID_ARG, "null argument");
    if (m->members != 1) return err(WEDGE_ERR_UNSUPPORTED, "gradients are defined for one-member models");
    wedge_status st = model_to_device(m);
    if (st != WEDGE_OK) return st;
    DevBuf dx, dt, dm, dg, dl;
    SetupLock alloc_lock;
    HTRY(hipMalloc(&dx.p, (size_t)count * kMlpIn * 4), "grad buffers");
    HTRY(hipMalloc(&dt.p, (size_t)count * kMlpOut * 4), "grad buffers");
    HTRY(hipMalloc(&dm.p, (size_t)count * kMlpOut * 4), "grad buffers");
    HTRY(hipMalloc(&dg.p, kMlpParams * 4), "grad buffers");
    HTRY(hipMalloc(&dl.p, 4), "grad buffers");
    HTRY(hipMemcpyAsync(dx.p, x, (size_t)count * kMlpIn * 4, hipMemcpyHostToDevice, stream), "upload");
    HTRY(hipMemcpyAsync(dt.p, t, (size_t)count * kMlpOut * 4, hipMemcpyHostToDevice, stream), "upload");
    HTRY(hipMemcpyAsync(dm.p, mask, (size_t)count * kMlpOut * 4, hipMemcpyHostToDevice, stream), "upload");
    HTRY(hipMemsetAsync(dg.p, 0, kMlpParams * 4, stream), "clear");
    HTRY(hipMemsetAsync(dl.p, 0, 4, stream), "clear");
    HTRY(launch_mlp_grad(m->dev_params, (const float*)dx.p, (const float*)dt.p, (const float*)dm.p, count,
                         1.0f / (float)count, (float*)dg.p, (float*)dl.p, stream), "gradient");
    HTRY(hipMemcpyAsync(grad, dg.p, kMlpParams * 4, hipMemcpyDeviceToHost, stream), "download");
    if (loss) HTRY(hipMemcpyAsync(loss, dl.p, 4, hipMemcpyDeviceToHost, stream), "download");
    HTRY(hipStreamSynchronize(stream), "gradient");
    return WEDGE_OK;
}

wedge_status wedge_model_train(wedge_model_t m, const wedge_trace_sample* s, uint32_t count,
                               uint32_t epochs, float lr, hipStream_t stream, float* final_loss) {
    if (!m || !s || !count) return err(WEDGE_ERR_INVALID_ARG, "null argument or no samples");
    if (!(lr > 0.f)) return err(WEDGE_ERR_INVALID_ARG, "lr must be > 0");
    std::vector<float> X((size_t)count * kMlpIn), T((size_t)count * kMlpOut), M((size_t)count * kMlpOut);
    wedge_model_features(s, count, X.data());
    // targets relative to the full pull of the same iteration: only differences
    // between modes decide, and they carry over across graph sizes far better
    // than absolute times
    for (uint32_t i = 0; i < count; ++i) {
        const double ref = s[i].t_us[0] > 0.f ? std::log1p((double)s[i].t_us[0]) : 0.0;
        for (int j = 0; j < kMlpOut; ++j) {
            const float tu = s[i].t_us[j];
            const bool ok = tu > 0.f && s[i].t_us[0] > 0.f;
            M[(size_t)i * kMlpOut + j] = ok ? 1.f : 0.f;
            T[(size_t)i * kMlpOut + j] = ok ? (float)(std::log1p((double)tu) - ref) : 0.f;
        }
    }
    // training envelope: per-feature range widened by 5% on each side, for the
    // scale-free features only; graph size (4) and the previous time (6) are
    // left open so a model trained on small graphs serves larger ones
    for (int f = 0; f < kMlpIn; ++f) {
        if (f == 4 || f == 6) {
            m->lo[f] = -std::numeric_limits<float>::infinity();
            m->hi[f] = std::numeric_limits<float>::infinity();
            continue;
        }
        float lo = std::numeric_limits<float>::infinity(), hi = -lo;
        for (uint32_t i = 0; i < count; ++i) {
            lo = std::fmin(lo, X[(size_t)i * kMlpIn + f]);
            hi = std::fmax(hi, X[(size_t)i * kMlpIn + f]);
        }
        const float pad = 0.05f * (hi - lo) + 1e-6f;
        m->lo[f] = lo - pad;
        m->hi[f] = hi + pad;
    }
    m->dirty = true;
    wedge_status st = model_to_device(m);
    if (st != WEDGE_OK) return st;
    DevBuf dx, dt, dm, dg, d1, d2, dl;
    SetupLock alloc_lock;
    HTRY(hipMalloc(&dx.p, X.size() * 4), "training buffers");
    HTRY(hipMalloc(&dt.p, T.size() * 4), "training buffers");
    HTRY(hipMalloc(&dm.p, M.size() * 4), "training buffers");
    HTRY(hipMalloc(&dg.p, kMlpParams * 4), "training buffers");
    HTRY(hipMalloc(&d1.p, kMlpParams * 4), "training buffers");
    HTRY(hipMalloc(&d2.p, kMlpParams * 4), "training buffers");
    HTRY(hipMalloc(&dl.p, 4), "training buffers");
    HTRY(hipMemcpyAsync(dx.p, X.data(), X.size() * 4, hipMemcpyHostToDevice, stream), "upload");
    HTRY(hipMemcpyAsync(dt.p, T.data(), T.size() * 4, hipMemcpyHostToDevice, stream), "upload");
    HTRY(hipMemcpyAsync(dm.p, M.data(), M.size() * 4, hipMemcpyHostToDevice, stream), "upload");
    // each member is trained on its own from its own initial parameters (Adam
    // state restarts per member); the reported loss is the members' mean
    float lsum = 0.f;
    for (uint32_t mb = 0; mb < m->members; ++mb) {
        float* P = m->dev_params + (size_t)mb * kMlpParams;
        HTRY(hipMemsetAsync(dg.p, 0, kMlpParams * 4, stream), "clear");
        HTRY(hipMemsetAsync(d1.p, 0, kMlpParams * 4, stream), "clear");
        HTRY(hipMemsetAsync(d2.p, 0, kMlpParams * 4, stream), "clear");
        for (uint32_t e = 0; e < epochs; ++e) {
            const bool last = e + 1 == epochs;
            if (last) HTRY(hipMemsetAsync(dl.p, 0, 4, stream), "clear");
            HTRY(launch_mlp_grad(P, (const float*)dx.p, (const float*)dt.p, (const float*)dm.p, count,
                                 1.0f / (float)count, (float*)dg.p, last ? (float*)dl.p : nullptr,
                                 stream), "gradient");
            HTRY(launch_adam(P, (float*)dg.p, (float*)d1.p, (float*)d2.p, lr, 0.9f, 0.999f, 1e-8f, e + 1,
                             stream), "adam");
        }
        float l = 0.f;
        HTRY(hipMemcpyAsync(&l, dl.p, 4, hipMemcpyDeviceToHost, stream), "download");
        HTRY(hipStreamSynchronize(stream), "training");
        lsum += l;
    }
    HTRY(hipMemcpyAsync(m->params.data(), m->dev_params, (size_t)m->members * kMlpParams * 4,
                        hipMemcpyDeviceToHost, stream), "download");
    HTRY(hipStreamSynchronize(stream), "training");
    if (final_loss) *final_loss = lsum / (float)m->members;
    return WEDGE_OK;
}

}  // extern "C"
