// HIP kernels of the expanding-channel vielbein LB path (gfx950, FP64).
//
// Busuioc & Ambrus, arXiv:1708.05944, Sec. VI: the reduced BGK equation in the
// coordinates (lambda, xi) with the orthonormal triad of Sec. VI.A, in conservative
// form with respect to (lambda, chi^xi) (Eqs. canalie_boltz, canalie_V, chi_canalie).
// One launch = one RK3 stage (Sec. III.A, Eq. rk3) for every cell of every instance.
// A block owns one cell and one distribution (f' or f''), one thread per velocity:
//   * FP64 block sums of the cell's moments (Sec. IV.A) -> n, u, T, tau = Kn/(nT)
//     (Eq. canalie_tau) and the polynomial equilibrium (Sec. IV.D);
//   * for cells within three of a wall, the wall density n_w of its xi column from the
//     wall-bound WENO flux (Sec. VI.B.4 with Eq. nw, applied at lambda = -1 and +1);
//   * epsilon-free WENO-5 face values (Sec. III.C) on both lambda faces (upwinded by
//     the sign of p^lambda) and both xi faces (upwinded by the sign of V^xi, which
//     varies with the face and the velocity), reservoir ghosts at the channel ends;
//   * the two connection terms with the four projected momentum derivatives
//     (Sec. IV.C kernels) from an LDS copy of the cell's populations;
//   * BGK, the Shu-Osher combination, and FP64 residual partials when asked.
#include <hip/hip_runtime.h>

#include "channel_internal.h"
#include "vlb_device.h"
#include "vlb_internal.h"

namespace vlb {

namespace {

constexpr int kChanThreads = kMaxNV;   // upper bound of the block size (NV rounded to 64)

// NQ sums over all threads of the block, in a fixed order (wavefront DPP sums, then the
// wavefront totals in wavefront order); every thread receives the totals.  sh holds
// 16 NQ doubles.
template <int NQ>
__device__ __forceinline__ void block_sums(double (&v)[NQ], double* sh) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double t = wave_sum(v[q]);
        if (lane == 0) sh[wave * NQ + q] = t;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double a = 0.0;
        for (int w = 0; w < nw; ++w) a += sh[w * NQ + q];
        v[q] = a;
    }
    __syncthreads();
}

__device__ __forceinline__ int find_instance(const long long* base, int B, long long b) {
    int i = 0;
    while (i + 1 < B && base[i + 1] <= b) ++i;
    return i;
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kChanThreads) void channel_stage(ChanArgs A) {
    __shared__ double sh[16 * 5];
    __shared__ double ecoef[kEqStride];
    __shared__ double gfac[kWave];
    __shared__ T row[kMaxNV];

    const long long b = blockIdx.x;
    const int inst = find_instance(A.base, A.B, b);
    const ChanDesc& I = A.inst[inst];
    const int NL = I.NL, NX = I.NX, NV = I.NV, Q1 = I.Q1, Q2 = I.Q2;
    const int ncell = NX * NL;
    const long long loc = b - A.base[inst];
    const int d = (int)(loc / ncell);
    const int cell = (int)(loc - (long long)d * ncell);
    const int p = cell / NL, s = cell - p * NL;
    const double* tab = A.tab + I.offT;
    const int k = threadIdx.x;
    const bool act = k < NV;
    const int kk = act ? k : 0, vi = kk / Q2, vj = kk - vi * Q2;
    const double pl = tab[I.tp1 + vi], px = tab[I.tp2 + vj];
    const T* F = static_cast<const T*>(A.Fin) + I.offF;
    auto at = [&](int dd, int pp, int ss) -> const T* { return F + (((size_t)dd * NX + pp) * NL + ss) * NV; };
    const T eps = T(I.weno_eps);

    // ---- moments of the cell (both distributions)
    double m[5];
    {
        const double f0 = act ? (double)at(0, p, s)[k] : 0.0, f1 = act ? (double)at(1, p, s)[k] : 0.0;
        m[0] = f0;
        m[1] = pl * f0;
        m[2] = px * f0;
        m[3] = (pl * pl + px * px) * f0;
        m[4] = f1;
    }
    block_sums<5>(m, sh);

    // ---- wall densities of this xi column (lambda = -1: emitted p^lambda > 0; +1: < 0)
    double nw_lo = 0.0, nw_hi = 0.0;
    const bool near_lo = s < 3, near_hi = s >= NL - 3;
    if (near_lo || near_hi) {
        double w[2] = {0.0, 0.0};
        if (act && near_lo && pl < 0) {
            const T F1 = at(0, p, 0)[k], F2 = at(0, p, 1)[k], F3 = at(0, p, 2)[k];
            const T g0 = T(3) * F1 - T(3) * F2 + F3, gm1 = T(6) * F1 - T(8) * F2 + T(3) * F3;
            w[0] = pl * (double)weno5<T>(F3, F2, F1, g0, gm1, eps);
        }
        if (act && near_hi && pl > 0) {
            const T G1 = at(0, p, NL - 1)[k], G2 = at(0, p, NL - 2)[k], G3 = at(0, p, NL - 3)[k];
            const T g0 = T(3) * G1 - T(3) * G2 + G3, gp1 = T(6) * G1 - T(8) * G2 + T(3) * G3;
            w[1] = pl * (double)weno5<T>(G3, G2, G1, g0, gp1, eps);
        }
        block_sums<2>(w, sh);
        nw_lo = -w[0] / I.den_lo;
        nw_hi = -w[1] / I.den_hi;
    }

    // ---- equilibrium of the cell, and its populations in LDS for the force terms
    if (threadIdx.x == 0) {
        const double n = m[0], u1 = m[1] / n, u2 = m[2] / n;
        const double T_ = (m[3] + m[4] - n * (u1 * u1 + u2 * u2)) / (3.0 * n);
        ecoef[0] = n;
        ecoef[1] = T_;
        ecoef[2] = 1.0 / tau_of(I.tau_model, I.Kn, n, T_);
        axis_coef(I.kind1, I.N1, u1, T_, tab + I.tC1, tab + I.tisf1, ecoef + 3, ecoef + 3 + (I.N1 + 1));
        axis_coef(I.kind2, I.N2, u2, T_, tab + I.tC2, tab + I.tisf2, ecoef + 3 + 2 * (I.N1 + 1),
                  ecoef + 3 + 2 * (I.N1 + 1) + (I.N2 + 1));
    }
    const T Fc = act ? at(d, p, s)[k] : T(0);
    if (act) row[k] = Fc;
    __syncthreads();
    if (threadIdx.x < Q1 + Q2) {
        const bool ax1 = threadIdx.x < Q1;
        const int node = ax1 ? threadIdx.x : threadIdx.x - Q1;
        const int nb = ax1 ? I.N1 + 1 : I.N2 + 1;
        const double* brow = tab + (ax1 ? I.tB1 : I.tB2) + node * nb;
        const int coff = ax1 ? 3 + ((I.kind1 == 1 && node >= I.Qh1) ? nb : 0)
                             : 3 + 2 * (I.N1 + 1) + ((I.kind2 == 1 && node >= I.Qh2) ? nb : 0);
        double g = 0.0;
        for (int l = 0; l < nb; ++l) g += brow[l] * ecoef[coff + l];
        gfac[threadIdx.x] = g;
    }
    __syncthreads();

    double rd = 0.0, rn = 0.0;
    T out = T(0);
    if (act) {
        // lambda stencil of column p: walls at both ends
        const double fw = tab[I.tfw + d * NV + k];
        auto lam_cell = [&](int c) -> T {
            if (c >= 0 && c < NL) return at(d, p, c)[k];
            if (c < 0) {
                if (pl > 0) return T(nw_lo * fw);                         // Eq. weno_populate
                const T F1 = at(d, p, 0)[k], F2 = at(d, p, 1)[k], F3 = at(d, p, 2)[k];
                if (c == -1) return T(3) * F1 - T(3) * F2 + F3;           // Eq. extrapol
                if (c == -2) return T(6) * F1 - T(8) * F2 + T(3) * F3;
                return T(0);
            }
            if (pl < 0) return T(nw_hi * fw);
            const T G1 = at(d, p, NL - 1)[k], G2 = at(d, p, NL - 2)[k], G3 = at(d, p, NL - 3)[k];
            if (c == NL) return T(3) * G1 - T(3) * G2 + G3;
            if (c == NL + 1) return T(6) * G1 - T(8) * G2 + T(3) * G3;
            return T(0);
        };
        T lw[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) lw[q] = lam_cell(s - 3 + q);
        T Fl, Fr;
        if (pl > 0) {
            Fl = weno5<T>(lw[0], lw[1], lw[2], lw[3], lw[4], eps);
            Fr = weno5<T>(lw[1], lw[2], lw[3], lw[4], lw[5], eps);
        } else {
            Fl = weno5<T>(lw[5], lw[4], lw[3], lw[2], lw[1], eps);
            Fr = weno5<T>(lw[6], lw[5], lw[4], lw[3], lw[2], eps);
        }
        // xi stencil of row s: reservoir Maxwellian for entering, the end cell for leaving
        const double* xc = tab + I.txc;
        const double* xa = tab + I.txa;
        const double vin = xc[s] * (px - xa[s] * pl);
        const double vout = xc[(size_t)NX * NL + s] * (px - xa[(size_t)NX * NL + s] * pl);
        auto xi_cell = [&](int c) -> T {
            if (c >= 0 && c < NX) return at(d, c, s)[k];
            if (c < 0) return vin > 0 ? T(tab[I.tfin + d * NV + k]) : at(d, 0, s)[k];
            return vout < 0 ? T(tab[I.tfout + d * NV + k]) : at(d, NX - 1, s)[k];
        };
        T xw[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) xw[q] = (q < 7) ? xi_cell(p - 3 + q) : T(0);
        double Vx[2];
        T Fx[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int f = p + e;   // face between cells f - 1 and f; stencil index of cell c is c - p + 3
            Vx[e] = xc[(size_t)f * NL + s] * (px - xa[(size_t)f * NL + s] * pl);
            Fx[e] = Vx[e] > 0 ? weno5<T>(xw[e], xw[e + 1], xw[e + 2], xw[e + 3], xw[e + 4], eps)
                              : weno5<T>(xw[e + 5], xw[e + 4], xw[e + 3], xw[e + 2], xw[e + 1], eps);
        }
        const double al = tab[I.tal + cell], ar = tab[I.tar + cell];
        const double adv_l = pl * (ar * (double)Fr - al * (double)Fl) / tab[I.tdlam + s];
        const double adv_x = (Vx[1] * (double)Fx[1] - Vx[0] * (double)Fx[0]) / tab[I.tdchi + p];
        // momentum derivatives (Sec. IV.C) along p^lambda (i) and p^xi (j)
        double k1 = 0.0, kt1 = 0.0, k2 = 0.0, kt2 = 0.0;
        for (int ip = 0; ip < Q1; ++ip) {
            const double r_ = (double)row[ip * Q2 + vj];
            k1 += tab[I.tK1 + vi * Q1 + ip] * r_;
            kt1 += tab[I.tKt1 + vi * Q1 + ip] * r_;
        }
        for (int jp = 0; jp < Q2; ++jp) {
            const double r_ = (double)row[vi * Q2 + jp];
            k2 += tab[I.tK2 + vj * Q2 + jp] * r_;
            kt2 += tab[I.tKt2 + vj * Q2 + jp] * r_;
        }
        const double glxx = tab[I.tglxx + cell], gxll = -tab[I.tglxl + cell];
        const double force = glxx * (px * px * k1 - pl * kt2) + gxll * (pl * pl * k2 - px * kt1);
        double fe = ecoef[0] * gfac[vi] * gfac[Q1 + vj];
        if (d) fe *= ecoef[1];
        const double L = -adv_l - adv_x + force - ((double)Fc - fe) * ecoef[2];
        if (A.l_only) {
            out = T(L);
        } else {
            const size_t idx = (((size_t)d * NX + p) * NL + s) * NV + k;
            const T fn = A.ca != 0.0 ? (static_cast<const T*>(A.Fn) + I.offF)[idx] : T(0);
            out = T(A.ca) * fn + T(A.cb) * Fc + T(A.cc * I.dt) * T(L);
            const double iw = tab[I.tiW + k];
            rd = ((double)out - (double)fn) * ((double)out - (double)fn) * iw;
            rn = (double)fn * (double)fn * iw;
        }
        (static_cast<T*>(A.Fout) + I.offF)[(((size_t)d * NX + p) * NL + s) * NV + k] = out;
    }
    if (A.rpart) {
        double r[2] = {rd, rn};
        block_sums<2>(r, sh);
        if (threadIdx.x == 0) {
            const double vol = tab[I.tvol + cell];
            A.rpart[((size_t)(I.offC + cell) * 2 + d) * 2] = vol * r[0];
            A.rpart[((size_t)(I.offC + cell) * 2 + d) * 2 + 1] = vol * r[1];
        }
    }
}

// Residual per instance: sqrt(sum of weighted squared changes / sum of weighted squares)
// / dt over every cell and both distributions, one block per instance, fixed order.
__global__ __launch_bounds__(256) void channel_reduce(const ChanDesc* insts, const double* tab_all,
                                                      const double* rpart, double* resid) {
    __shared__ double sh[2][256];
    const ChanDesc& I = insts[blockIdx.x];
    const int t = threadIdx.x, nc = I.NX * I.NL;
    double a = 0.0, c = 0.0;
    for (int x = t; x < 2 * nc; x += 256) {
        const double* rp = rpart + ((size_t)I.offC * 2 + x) * 2;
        a += rp[0];
        c += rp[1];
    }
    sh[0][t] = a;
    sh[1][t] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) { sh[0][t] += sh[0][t + w]; sh[1][t] += sh[1][t + w]; }
        __syncthreads();
    }
    if (t == 0) resid[blockIdx.x] = sqrt(sh[0][0] / sh[1][0]) / I.dt;
}

// n, u^lambda, u^xi, T and the particle content vol * n of every cell.
__global__ __launch_bounds__(kChanThreads) void channel_diag(const ChanDesc* insts, const long long* cbase, int B,
                                                             const double* tab_all, const double* F, double* diag) {
    __shared__ double sh[16 * 5];
    const long long b = blockIdx.x;
    const int inst = find_instance(cbase, B, b);
    const ChanDesc& I = insts[inst];
    const int cell = (int)(b - cbase[inst]);
    const double* tab = tab_all + I.offT;
    const int k = threadIdx.x, NV = I.NV;
    const bool act = k < NV;
    const int kk = act ? k : 0, vi = kk / I.Q2, vj = kk - vi * I.Q2;
    const double pl = tab[I.tp1 + vi], px = tab[I.tp2 + vj];
    const double* f = F + I.offF + (size_t)cell * NV;
    const size_t dsz = (size_t)I.NX * I.NL * NV;
    const double f0 = act ? f[k] : 0.0, f1 = act ? f[dsz + k] : 0.0;
    double m[5] = {f0, pl * f0, px * f0, (pl * pl + px * px) * f0, f1};
    block_sums<5>(m, sh);
    if (threadIdx.x == 0) {
        const double n = m[0], u1 = m[1] / n, u2 = m[2] / n;
        double* o = diag + (size_t)(I.offC + cell) * 5;
        o[0] = n;
        o[1] = u1;
        o[2] = u2;
        o[3] = (m[3] + m[4] - n * (u1 * u1 + u2 * u2)) / (3.0 * n);
        o[4] = tab[I.tvol + cell] * n;
    }
}

hipError_t launch_channel_stage(long long nblocks, int threads, hipStream_t st, const ChanArgs& A) {
    hipLaunchKernelGGL(channel_stage<double>, dim3((unsigned)nblocks), dim3(threads), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_channel_reduce(int ninst, hipStream_t st, const ChanDesc* insts, const double* tab,
                                 const double* rpart, double* resid) {
    hipLaunchKernelGGL(channel_reduce, dim3(ninst), dim3(256), 0, st, insts, tab, rpart, resid);
    return hipGetLastError();
}

hipError_t launch_channel_diag(long long ncells_total, int threads, hipStream_t st, const ChanDesc* insts,
                               const long long* cbase, int B, const double* tab, const double* F, double* diag) {
    hipLaunchKernelGGL(channel_diag, dim3((unsigned)ncells_total), dim3(threads), 0, st, insts, cbase, B, tab, F,
                       diag);
    return hipGetLastError();
}

}  // namespace vlb
