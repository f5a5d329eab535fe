// Host side of the warm-start surrogate: parameter storage, Adam state, activation
// buffers and the enqueueing of the layer products (mlp_kernels.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "mlp_internal.h"

using namespace vlb;

struct vlb_mlp {
    int width = 0, depth = 0;
    std::vector<int> fin, fout;          // per layer
    std::vector<size_t> woff, boff;      // parameter offsets per layer
    size_t nparam = 0;
    hipStream_t stream = nullptr;
    float *theta = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
    long t = 0;                          // Adam steps taken
    bool have_grad = false;
    // activation buffers for up to cap rows: Z[depth], H[depth], Y, G (two), Xb, Tb
    long cap = 0;
    float* act = nullptr;
    float *Z0 = nullptr, *H0 = nullptr, *Y = nullptr, *Ga = nullptr, *Gb = nullptr, *Xb = nullptr, *Tb = nullptr;
    float* part = nullptr;               // split-K partials / loss partials
    size_t part_cap = 0;
    float* loss = nullptr;               // per-step losses of the last train call
    long loss_cap = 0;
    int* idx = nullptr;
    long idx_cap = 0;

    float* Z(int l) { return Z0 + (size_t)l * cap * width; }
    float* H(int l) { return H0 + (size_t)l * cap * width; }
};

namespace {

constexpr float kB1 = 0.9f, kB2 = 0.999f, kEps = 1e-8f;
constexpr int kSplitRows = 256;   // batch rows per split of a weight-gradient product

vlb_status grow(void** p, size_t bytes) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return set_error(VLB_ENOMEM, "hipMalloc(%zu) failed", bytes);
    }
    return VLB_OK;
}

vlb_status ensure_rows(vlb_mlp* m, long rows) {
    if (rows <= m->cap) return VLB_OK;
    VLB_HIP_TRY(hipStreamSynchronize(m->stream));
    const long cap = std::max(rows, 2 * m->cap);
    const size_t per = (size_t)cap;
    const size_t n = per * m->width * (2 * m->depth + 2) + per * (kMlpOut + kMlpIn + kMlpOut);
    vlb_status s = grow((void**)&m->act, n * sizeof(float));
    if (s != VLB_OK) { m->cap = 0; return s; }
    m->cap = cap;
    float* p = m->act;
    m->Z0 = p; p += per * m->width * m->depth;
    m->H0 = p; p += per * m->width * m->depth;
    m->Ga = p; p += per * m->width;
    m->Gb = p; p += per * m->width;
    m->Y = p; p += per * kMlpOut;
    m->Xb = p; p += per * kMlpIn;
    m->Tb = p;
    return VLB_OK;
}

vlb_status ensure_part(vlb_mlp* m, size_t n) {
    if (n <= m->part_cap) return VLB_OK;
    VLB_HIP_TRY(hipStreamSynchronize(m->stream));
    const size_t cap = std::max(n, 2 * m->part_cap);
    vlb_status s = grow((void**)&m->part, cap * sizeof(float));
    m->part_cap = s == VLB_OK ? cap : 0;
    return s;
}

// Forward pass on n rows of X (layer inputs kept for the backward pass when train).
vlb_status forward(vlb_mlp* m, const float* X, long n, float* Y, bool bf16, bool train, hipStream_t st) {
    const float* in = X;
    for (int l = 0; l <= m->depth; ++l) {
        GemmArgs g{};
        g.A = in;
        g.as_m = m->fin[l];
        g.as_k = 1;
        g.B = m->theta + m->woff[l];
        g.bs_k = m->fout[l];
        g.bs_n = 1;
        g.M = (int)n;
        g.N = m->fout[l];
        g.K = m->fin[l];
        g.kchunk = g.K;
        g.bias = m->theta + m->boff[l];
        g.cs_m = m->fout[l];
        int epi;
        if (l == m->depth) {
            g.C = Y;
            epi = kEpiBias;
        } else {
            // inference ping-pongs between two hidden buffers; training keeps every layer
            g.C = train ? m->Z(l) : nullptr;
            g.H = train ? m->H(l) : m->H(l & 1);
            epi = kEpiBiasSilu;
            in = g.H;
        }
        VLB_HIP_TRY(launch_mlp_gemm(epi, bf16, g, 1, st));
    }
    return VLB_OK;
}

// Loss and gradient of rows (X, T) already in the activation buffers' row space.
vlb_status loss_grad(vlb_mlp* m, const float* X, const float* T, long n, float* loss_dst) {
    hipStream_t st = m->stream;
    vlb_status s = forward(m, X, n, m->Y, false, true, st);
    if (s != VLB_OK) return s;
    const long nout = n * kMlpOut;
    const int nsplit = (int)((n + kSplitRows - 1) / kSplitRows);
    size_t need = (size_t)((nout + 255) / 256);
    for (int l = 0; l <= m->depth; ++l) need = std::max(need, (size_t)nsplit * m->fin[l] * m->fout[l]);
    s = ensure_part(m, need);
    if (s != VLB_OK) return s;
    VLB_HIP_TRY(launch_mlp_loss(m->Y, T, nout, 2.0f / (float)nout, m->Ga, m->part, loss_dst, st));
    float* G = m->Ga;
    float* Gn = m->Gb;
    for (int l = m->depth; l >= 0; --l) {
        const float* in = l ? m->H(l - 1) : X;
        GemmArgs g{};   // dW_l = in^T G, split over the batch
        g.A = in;
        g.as_m = 1;
        g.as_k = m->fin[l];
        g.B = G;
        g.bs_k = m->fout[l];
        g.bs_n = 1;
        g.M = m->fin[l];
        g.N = m->fout[l];
        g.K = (int)n;
        g.kchunk = kSplitRows;
        g.C = m->part;
        g.cs_m = m->fout[l];
        VLB_HIP_TRY(launch_mlp_gemm(kEpiStore, false, g, nsplit, st));
        VLB_HIP_TRY(launch_mlp_splitk_sum(m->part, nsplit, (long)m->fin[l] * m->fout[l], m->grad + m->woff[l], st));
        VLB_HIP_TRY(launch_mlp_colsum(G, (int)n, m->fout[l], m->grad + m->boff[l], st));
        if (l == 0) break;
        GemmArgs h{};   // G_{l-1} = (G W_l^T) * silu'(Z_{l-1})
        h.A = G;
        h.as_m = m->fout[l];
        h.as_k = 1;
        h.B = m->theta + m->woff[l];
        h.bs_k = 1;
        h.bs_n = m->fout[l];
        h.M = (int)n;
        h.N = m->fin[l];
        h.K = m->fout[l];
        h.kchunk = h.K;
        h.Z = m->Z(l - 1);
        h.C = Gn;
        h.cs_m = m->fin[l];
        VLB_HIP_TRY(launch_mlp_gemm(kEpiDsilu, false, h, 1, st));
        std::swap(G, Gn);
    }
    m->have_grad = true;
    return VLB_OK;
}

vlb_status adam(vlb_mlp* m, float lr) {
    m->t += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)kB1, (double)m->t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)kB2, (double)m->t)));
    VLB_HIP_TRY(launch_mlp_adam(m->theta, m->m1, m->m2, m->grad, (long)m->nparam, lr, kB1, kB2, kEps, c1, c2,
                                m->stream));
    return VLB_OK;
}

size_t count_params(int width, int depth) {
    size_t n = 0;
    for (int l = 0; l <= depth; ++l) {
        const size_t a = l ? width : kMlpIn, b = l == depth ? kMlpOut : width;
        n += a * b + b;
    }
    return n;
}

bool shape_ok(int width, int depth) { return width >= 1 && width <= 1024 && depth >= 1 && depth <= 8; }

}  // namespace

namespace vlb {

vlb_status mlp_infer(vlb_mlp* m, const float* X, long n, float* Y, int bf16, hipStream_t st) {
    if (n <= 0) return VLB_OK;
    vlb_status s = ensure_rows(m, n);
    if (s != VLB_OK) return s;
    return forward(m, X, n, Y, bf16 != 0, false, st);
}

hipStream_t mlp_stream(const vlb_mlp* m) { return m->stream; }

}  // namespace vlb

extern "C" {

vlb_status vlb_mlp_param_count(int width, int depth, size_t* n) {
    if (!n || !shape_ok(width, depth)) return set_error(VLB_EINVAL, "width must be 1..1024 and depth 1..8");
    *n = count_params(width, depth);
    return VLB_OK;
}

vlb_status vlb_mlp_create(vlb_mlp** out, int width, int depth, const float* params, void* hip_stream) {
    if (!out || !params || !shape_ok(width, depth)) return set_error(VLB_EINVAL, "bad arguments");
    *out = nullptr;
    for (size_t i = 0, n = count_params(width, depth); i < n; ++i)
        if (!std::isfinite(params[i])) return set_error(VLB_ENONFINITE, "parameter %zu is not finite", i);
    vlb_mlp* m = new (std::nothrow) vlb_mlp;
    if (!m) return set_error(VLB_ENOMEM, "out of host memory");
    m->width = width;
    m->depth = depth;
    m->stream = (hipStream_t)hip_stream;
    size_t o = 0;
    for (int l = 0; l <= depth; ++l) {
        m->fin.push_back(l ? width : kMlpIn);
        m->fout.push_back(l == depth ? kMlpOut : width);
        m->woff.push_back(o);
        o += (size_t)m->fin[l] * m->fout[l];
        m->boff.push_back(o);
        o += m->fout[l];
    }
    m->nparam = o;
    void* p = nullptr;
    if (hipMalloc(&p, 4 * o * sizeof(float)) != hipSuccess) {
        delete m;
        return set_error(VLB_ENOMEM, "hipMalloc of %zu parameters failed", o);
    }
    m->theta = (float*)p;
    m->m1 = m->theta + o;
    m->m2 = m->m1 + o;
    m->grad = m->m2 + o;
    hipError_t e = hipMemcpyAsync(m->theta, params, o * sizeof(float), hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->m1, 0, 3 * o * sizeof(float), m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        (void)hipFree(p);
        delete m;
        return set_error(VLB_EDEVICE, "parameter upload failed: %s", hipGetErrorString(e));
    }
    *out = m;
    return VLB_OK;
}

vlb_status vlb_mlp_destroy(vlb_mlp* m) {
    if (!m) return VLB_OK;
    (void)hipStreamSynchronize(m->stream);
    for (void* p : {(void*)m->theta, (void*)m->act, (void*)m->part, (void*)m->loss, (void*)m->idx})
        if (p) (void)hipFree(p);
    delete m;
    return VLB_OK;
}

vlb_status vlb_mlp_get_params(vlb_mlp* m, float* host, size_t n) {
    if (!m || !host || n != m->nparam) return set_error(VLB_EINVAL, "parameter count mismatch");
    VLB_HIP_TRY(hipMemcpyAsync(host, m->theta, n * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    VLB_HIP_TRY(hipStreamSynchronize(m->stream));
    return VLB_OK;
}

vlb_status vlb_mlp_set_params(vlb_mlp* m, const float* host, size_t n) {
    if (!m || !host || n != m->nparam) return set_error(VLB_EINVAL, "parameter count mismatch");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return set_error(VLB_ENONFINITE, "parameter %zu is not finite", i);
    VLB_HIP_TRY(hipMemcpyAsync(m->theta, host, n * sizeof(float), hipMemcpyHostToDevice, m->stream));
    VLB_HIP_TRY(hipMemsetAsync(m->m1, 0, 3 * n * sizeof(float), m->stream));
    VLB_HIP_TRY(hipStreamSynchronize(m->stream));
    m->t = 0;
    m->have_grad = false;
    return VLB_OK;
}

vlb_status vlb_mlp_forward(vlb_mlp* m, const float* X, long n, float* Y, int bf16) {
    if (!m || n < 0 || (n > 0 && (!X || !Y))) return set_error(VLB_EINVAL, "bad arguments");
    return mlp_infer(m, X, n, Y, bf16, m->stream);
}

vlb_status vlb_mlp_loss_grad(vlb_mlp* m, const float* X, const float* T, long n, float* loss, float* grad) {
    if (!m || !X || !T || n <= 0 || n > (1L << 30)) return set_error(VLB_EINVAL, "bad arguments");
    vlb_status s = ensure_rows(m, n);
    if (s != VLB_OK) return s;
    if (!m->loss) {
        s = grow((void**)&m->loss, 1024 * sizeof(float));
        if (s != VLB_OK) return s;
        m->loss_cap = 1024;
    }
    s = loss_grad(m, X, T, n, m->loss);
    if (s != VLB_OK) return s;
    if (loss) VLB_HIP_TRY(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    if (grad) VLB_HIP_TRY(hipMemcpyAsync(grad, m->grad, m->nparam * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    VLB_HIP_TRY(hipStreamSynchronize(m->stream));
    return VLB_OK;
}

vlb_status vlb_mlp_adam_step(vlb_mlp* m, const float* grad, float lr) {
    if (!m || !(lr > 0) || !std::isfinite(lr)) return set_error(VLB_EINVAL, "bad arguments");
    if (grad) {
        VLB_HIP_TRY(hipMemcpyAsync(m->grad, grad, m->nparam * sizeof(float), hipMemcpyHostToDevice, m->stream));
    } else if (!m->have_grad) {
        return set_error(VLB_ESTATE, "no gradient computed yet");
    }
    vlb_status s = adam(m, lr);
    if (s != VLB_OK) return s;
    VLB_HIP_TRY(hipStreamSynchronize(m->stream));
    return VLB_OK;
}

vlb_status vlb_mlp_train(vlb_mlp* m, const float* X, const float* T, long nsamples, const int* order, long norder,
                         int batch, float lr, float* mean_loss) {
    if (!m || !X || !T || !order || nsamples <= 0 || norder <= 0 || batch <= 0 || batch > (1 << 20) ||
        !(lr > 0) || !std::isfinite(lr))
        return set_error(VLB_EINVAL, "bad arguments");
    for (long i = 0; i < norder; ++i)
        if (order[i] < 0 || order[i] >= nsamples) return set_error(VLB_EINVAL, "order[%ld] = %d out of range", i, order[i]);
    const long steps = (norder + batch - 1) / batch;
    vlb_status s = ensure_rows(m, std::min<long>(batch, norder));
    if (s != VLB_OK) return s;
    if (steps > m->loss_cap) {
        s = grow((void**)&m->loss, steps * sizeof(float));
        if (s != VLB_OK) { m->loss_cap = 0; return s; }
        m->loss_cap = steps;
    }
    if (norder > m->idx_cap) {
        VLB_HIP_TRY(hipStreamSynchronize(m->stream));
        s = grow((void**)&m->idx, norder * sizeof(int));
        if (s != VLB_OK) { m->idx_cap = 0; return s; }
        m->idx_cap = norder;
    }
    VLB_HIP_TRY(hipMemcpyAsync(m->idx, order, norder * sizeof(int), hipMemcpyHostToDevice, m->stream));
    for (long st = 0; st < steps; ++st) {
        const long r0 = st * batch;
        const int nb = (int)std::min<long>(batch, norder - r0);
        VLB_HIP_TRY(launch_mlp_gather(X, T, m->idx + r0, nb, kMlpIn, kMlpOut, m->Xb, m->Tb, m->stream));
        s = loss_grad(m, m->Xb, m->Tb, nb, m->loss + st);
        if (s != VLB_OK) return s;
        s = adam(m, lr);
        if (s != VLB_OK) return s;
    }
    if (mean_loss) {
        std::vector<float> h(steps);
        VLB_HIP_TRY(hipMemcpyAsync(h.data(), m->loss, steps * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        VLB_HIP_TRY(hipStreamSynchronize(m->stream));
        double acc = 0;
        for (float v : h) acc += v;
        *mean_loss = (float)(acc / steps);
    } else {
        VLB_HIP_TRY(hipStreamSynchronize(m->stream));
    }
    return VLB_OK;
}

}  // extern "C"
