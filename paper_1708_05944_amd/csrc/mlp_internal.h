// Internal declarations shared by the host sources of libvlb.so: the error channel of
// the C ABI and the surrogate network (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "../../include/vlb.h"

namespace vlb {

// Sets the thread-local message returned by vlb_last_error and returns s.
vlb_status set_error(vlb_status s, const char* fmt, ...);

#define VLB_HIP_TRY(expr)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return ::vlb::set_error(VLB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

enum { kEpiStore = 0, kEpiBias = 1, kEpiBiasSilu = 2, kEpiDsilu = 3 };

// Operands of one layer product C = A B: A(m, k) = A[m as_m + k as_k],
// B(k, n) = B[k bs_k + n bs_n], C(m, n) = C[m cs_m + n] (+ z M cs_m for the split-K
// partial z); bias[n], pre-activations Z (same shape as C, for SiLU'), H = silu(C).
struct GemmArgs {
    const float* A;
    long as_m, as_k;
    const float* B;
    long bs_k, bs_n;
    int M, N, K, kchunk;
    const float* bias;
    const float* Z;
    float* C;
    long cs_m;
    float* H;
};

hipError_t launch_mlp_gemm(int epi, bool bf16, const GemmArgs& g, int nsplit, hipStream_t st);
hipError_t launch_mlp_splitk_sum(const float* part, int nsplit, long n, float* out, hipStream_t st);
hipError_t launch_mlp_colsum(const float* G, int rows, int cols, float* out, hipStream_t st);
hipError_t launch_mlp_loss(const float* Y, const float* T, long n, float scale, float* G, float* part, float* dst,
                           hipStream_t st);
hipError_t launch_mlp_gather(const float* X, const float* T, const int* idx, int nb, int dx, int dt, float* Xb,
                             float* Tb, hipStream_t st);
hipError_t launch_mlp_adam(float* theta, float* m, float* v, const float* g, long n, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t st);

// Surrogate input and output widths.
constexpr int kMlpIn = 4, kMlpOut = 4;

// Inference of the network on n rows of X[n][4] into Y[n][4], enqueued on st.
vlb_status mlp_infer(vlb_mlp* m, const float* X, long n, float* Y, int bf16, hipStream_t st);
hipStream_t mlp_stream(const vlb_mlp* m);

}  // namespace vlb
