// Kernels of the warm-start surrogate: a SiLU multilayer perceptron trained by Adam.
//
// Every layer product runs on the matrix cores: FP32 operands with FP32 accumulation
// (v_mfma_f32_16x16x4_f32) for training, bfloat16 operands with FP32 accumulation
// (v_mfma_f32_16x16x16_bf16) for inference.  One kernel covers the three products of
// a layer (forward X W, weight gradient X^T G, input gradient G W^T) through operand
// strides, with the bias, SiLU and SiLU' epilogues fused; weight gradients split the
// batch dimension over blocks and are summed in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "mlp_internal.h"

namespace vlb {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = sigm(z);
    return s + z * s * (1.0f - s);
}

// nearest bfloat16 (ties to even) of a finite float, as raw bits
__device__ __forceinline__ short bf16_bits(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// C = A B with A(m, k) = A[m as_m + k as_k], B(k, n) = B[k bs_k + n bs_n].  A block of
// four wavefronts covers 64 rows x 16 columns (one 16 x 16 MFMA tile per wavefront);
// blockIdx.z takes rows [z kchunk, (z+1) kchunk) of the contraction.  Matrix-core
// lane layout (16 x 16 result): lane l holds C(4 (l/16) + i, l % 16), i = 0..3.
template <int EPI, bool BF16>
__global__ __launch_bounds__(256) void mlp_gemm(GemmArgs g) {
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int m0 = (blockIdx.x * 4 + wave) * 16, n0 = blockIdx.y * 16;
    if (m0 >= g.M) return;   // whole wavefront
    const int kb = blockIdx.z * g.kchunk, ke = min(g.K, kb + g.kchunk);
    const int r = l & 15, q = l >> 4;
    const int m = m0 + r, n = n0 + r;
    const bool mok = m < g.M, nok = n < g.N;
    const float* Ar = g.A + (long)(mok ? m : 0) * g.as_m;
    const float* Bc = g.B + (long)(nok ? n : 0) * g.bs_n;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (!BF16) {
        for (int k = kb; k < ke; k += 4) {
            const int kk = k + q;
            const float a = (mok && kk < ke) ? Ar[(long)kk * g.as_k] : 0.f;
            const float b = (nok && kk < ke) ? Bc[(long)kk * g.bs_k] : 0.f;
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
        }
    } else {
        for (int k = kb; k < ke; k += 16) {
            shortx4 a, b;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int kk = k + 4 * q + j;
                a[j] = bf16_bits((mok && kk < ke) ? Ar[(long)kk * g.as_k] : 0.f);
                b[j] = bf16_bits((nok && kk < ke) ? Bc[(long)kk * g.bs_k] : 0.f);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
    }
    if (!nok) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int mm = m0 + 4 * q + i;
        if (mm >= g.M) break;
        const long o = (long)mm * g.cs_m + n;
        float v = acc[i];
        if constexpr (EPI == kEpiStore) {
            g.C[(long)blockIdx.z * g.M * g.cs_m + o] = v;
        } else if constexpr (EPI == kEpiBias) {
            g.C[o] = v + g.bias[n];
        } else if constexpr (EPI == kEpiBiasSilu) {
            v += g.bias[n];
            if (g.C) g.C[o] = v;
            g.H[o] = silu(v);
        } else {
            g.C[o] = v * dsilu(g.Z[o]);
        }
    }
}

// out[i] = sum over z of part[z n + i], z in order
__global__ __launch_bounds__(256) void mlp_splitk_sum(const float* part, int nsplit, long n, float* out) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int z = 0; z < nsplit; ++z) s += part[(long)z * n + i];
    out[i] = s;
}

// out[c] = sum over rows of G[r cols + c]; one block per column, fixed-order tree
__global__ __launch_bounds__(256) void mlp_colsum(const float* G, int rows, int cols, float* out) {
    __shared__ float sh[256];
    const int c = blockIdx.x, t = threadIdx.x;
    float s = 0.f;
    for (int r = t; r < rows; r += 256) s += G[(long)r * cols + c];
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) out[c] = sh[0];
}

// G = scale (Y - T) over n values; part[block] = sum of (Y - T)^2 of the block's values
__global__ __launch_bounds__(256) void mlp_loss_grad(const float* Y, const float* T, long n, float scale, float* G,
                                                     float* part) {
    __shared__ float sh[256];
    const int t = threadIdx.x;
    const long i = (long)blockIdx.x * 256 + t;
    float d2 = 0.f;
    if (i < n) {
        const float d = Y[i] - T[i];
        G[i] = scale * d;
        d2 = d * d;
    }
    sh[t] = d2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = sh[0];
}

// dst[0] = inv_count * sum of part[0..nparts) (single block, fixed order)
__global__ __launch_bounds__(256) void mlp_sum_parts(const float* part, int nparts, float inv_count, float* dst) {
    __shared__ float sh[256];
    const int t = threadIdx.x;
    float s = 0.f;
    for (int i = t; i < nparts; i += 256) s += part[i];
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) dst[0] = sh[0] * inv_count;
}

// rows idx[r] of X[.][dx] and T[.][dt] gathered into Xb, Tb (indices checked on the host)
__global__ __launch_bounds__(256) void mlp_gather(const float* X, const float* T, const int* idx, int nb, int dx,
                                                  int dt, float* Xb, float* Tb) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= nb) return;
    const long s = idx[r];
    for (int j = 0; j < dx; ++j) Xb[(long)r * dx + j] = X[s * dx + j];
    for (int j = 0; j < dt; ++j) Tb[(long)r * dt + j] = T[s * dt + j];
}

// Adam with bias correction (c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t))
__global__ __launch_bounds__(256) void mlp_adam(float* theta, float* m, float* v, const float* g, long n, float lr,
                                                float b1, float b2, float eps, float c1, float c2) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ------------------------------------------------------------------ host launchers
hipError_t launch_mlp_gemm(int epi, bool bf16, const GemmArgs& g, int nsplit, hipStream_t st) {
    const dim3 grid((g.M + 63) / 64, (g.N + 15) / 16, nsplit), block(256);
    if (bf16) {
        if (epi == kEpiBias) hipLaunchKernelGGL((mlp_gemm<kEpiBias, true>), grid, block, 0, st, g);
        else if (epi == kEpiBiasSilu) hipLaunchKernelGGL((mlp_gemm<kEpiBiasSilu, true>), grid, block, 0, st, g);
        else return hipErrorInvalidValue;
    } else {
        if (epi == kEpiStore) hipLaunchKernelGGL((mlp_gemm<kEpiStore, false>), grid, block, 0, st, g);
        else if (epi == kEpiBias) hipLaunchKernelGGL((mlp_gemm<kEpiBias, false>), grid, block, 0, st, g);
        else if (epi == kEpiBiasSilu) hipLaunchKernelGGL((mlp_gemm<kEpiBiasSilu, false>), grid, block, 0, st, g);
        else hipLaunchKernelGGL((mlp_gemm<kEpiDsilu, false>), grid, block, 0, st, g);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_splitk_sum(const float* part, int nsplit, long n, float* out, hipStream_t st) {
    hipLaunchKernelGGL(mlp_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, nsplit, n, out);
    return hipGetLastError();
}

hipError_t launch_mlp_colsum(const float* G, int rows, int cols, float* out, hipStream_t st) {
    hipLaunchKernelGGL(mlp_colsum, dim3(cols), dim3(256), 0, st, G, rows, cols, out);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(const float* Y, const float* T, long n, float scale, float* G, float* part, float* dst,
                           hipStream_t st) {
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(mlp_loss_grad, dim3(nb), dim3(256), 0, st, Y, T, n, scale, G, part);
    hipLaunchKernelGGL(mlp_sum_parts, dim3(1), dim3(256), 0, st, part, nb, 1.0f / (float)n, dst);
    return hipGetLastError();
}

hipError_t launch_mlp_gather(const float* X, const float* T, const int* idx, int nb, int dx, int dt, float* Xb,
                             float* Tb, hipStream_t st) {
    hipLaunchKernelGGL(mlp_gather, dim3((nb + 255) / 256), dim3(256), 0, st, X, T, idx, nb, dx, dt, Xb, Tb);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* theta, float* m, float* v, const float* g, long n, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(mlp_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, theta, m, v, g, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

}  // namespace vlb
