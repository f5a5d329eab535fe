// HIP kernels of the expanding-channel vielbein LB path (gfx950, FP64).
//
// Busuioc & Ambrus, arXiv:1708.05944, Sec. VI: the reduced BGK equation in the
// coordinates (lambda, xi) with the orthonormal triad of Sec. VI.A, in conservative
// form with respect to (lambda, chi^xi) (Eqs. canalie_boltz, canalie_V, chi_canalie).
// One launch = one RK3 stage (Sec. III.A, Eq. rk3) for every cell of every instance of
// one velocity-tile class.  A wavefront owns one cell and both distributions (f', f'');
// a block is four independent wavefronts (four cells) and never synchronises.
//
// Velocities of a cell as 16 x 16 tiles of the (p^lambda node i, p^xi node j) grid,
// zero-padded to whole tiles.  Lane l = 16 g + n, register c of tile (I, J) holds
// i = 16 I + 4 c + g, j = 16 J + n.  With 16 p^xi nodes this is velocity k = 64 c + l:
// every load and store of a register moves 512 contiguous bytes.
//
// Per cell:
//   * FP64 wavefront sums of the cell's moments (Sec. IV.A) -> n, u, T and
//     tau = Kn/(nT) (Eq. canalie_tau); the polynomial equilibrium (Sec. IV.D);
//   * within three cells of a wall, the wall density n_w of the xi column from the
//     wall-bound WENO flux (Sec. VI.C.4 with Eq. nw, at lambda = -1 and +1);
//   * epsilon-free WENO-5 face values (Sec. III.C) on both lambda faces (upwinded by
//     the sign of p^lambda) and both xi faces (upwinded by the sign of V^xi, which
//     varies with the face and the velocity), reservoir ghosts at the channel ends;
//   * the four projected momentum derivatives (Sec. IV.C kernels) as FP64 16x16x4
//     MFMA products on the tiles, which land in the register layout above: the
//     derivatives along p^lambda contract the tile rows (F is the second operand, in its
//     own registers); those along p^xi contract the tile columns, with F as the first
//     operand read back through a wavefront-private LDS transpose;
//   * the two connection terms, BGK, the Shu-Osher combination and FP64 residual
//     partials when asked.
// Block b runs on XCD b mod 8; blocks are renumbered so that each XCD sweeps one
// contiguous band of cells and the xi-neighbour columns stay in its L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "channel_internal.h"
#include "vlb_device.h"
#include "vlb_internal.h"

namespace vlb {

namespace {

// order of the LDS operations of one wavefront (no cross-wavefront sharing)
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ int find_instance(const long long* base, int B, long long b) {
    int lo = 0, hi = B - 1;   // largest i with base[i] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// NQ sums over all threads of a block, in a fixed order (wavefront sums, then the
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

// Row order of the first MFMA operand that lands product row 4 r + g (the node of
// register r in lane group g) where the register layout wants it.  The FP64 16x16x4
// product holds row g + 4 r in register r of lane group g: already the wanted order.
// The FP32 16x16x4 product holds row 4 g + r there, so its operand rows are permuted by
// m -> 4 (m mod 4) + m / 4.
template <typename T>
__device__ __forceinline__ int mfma_row(int m);
template <>
__device__ __forceinline__ int mfma_row<double>(int m) { return m; }
template <>
__device__ __forceinline__ int mfma_row<float>(int m) { return 4 * (m & 3) + (m >> 2); }

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Acc4;
template <>
struct Acc4<double> {
    typedef dvec4 type;
    static __device__ __forceinline__ dvec4 mfma(double a, double b, dvec4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Acc4<float> {
    typedef fvec4 type;
    static __device__ __forceinline__ fvec4 mfma(float a, float b, fvec4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

}  // namespace

// T = double: populations f'_k, f''_k as stored (quadrature weights included).
// T = float: populations divided by W_k = w_i w_j (O(1) values); the tables of the FP32
// descriptor are rescaled to match (kernels diag(1/w) K diag(w), bases and ghost
// Maxwellians over w or W, residual weight W), and the moment and wall-flux sums
// multiply by W_k in FP64.
// BND = false: the interior cells (3 <= s < NL - 3, 3 <= p < NX - 3), whose stencils stay
// inside the grid, without any ghost logic; BND = true: the cells of the edge bands (walls,
// centreline, ends).  The two launches of a stage write disjoint cells.
template <typename T, int T1, int T2, bool BND>
__global__ __launch_bounds__(kChanWaves * kWave, T1 * T2 == 1 ? (sizeof(T) == 4 ? 4 : (BND ? 2 : 3))
                                                               : (sizeof(T) == 4 ? (BND ? 3 : 4) : 2)) void channel_stage(ChanArgs A) {
    constexpr bool F32 = sizeof(T) == 4;
    constexpr int NT = T1 * T2, NI = 4 * NT;   // items (tile registers) per lane per distribution
    constexpr int RS = 16 * T2 + 2;           // LDS row stride of the transpose buffer
    constexpr int S1 = 16 * T1 + 1, S2 = 16 * T2 + 1;   // LDS row strides of the kernel copies
    typedef typename Acc4<T>::type acc_t;
    __shared__ T k1s[16 * T1 * S1], kt1s[16 * T1 * S1], k2s[16 * T2 * S2], kt2s[16 * T2 * S2];
    __shared__ T trs[kChanWaves][16 * T1 * RS];   // F of the cell, [i][j] (this distribution)
    __shared__ T lcs[kChanWaves][16 * T1 * RS];   // L of the cell, [i][j]
    __shared__ double gsh[kChanWaves][kWave];
    __shared__ double ecs[kChanWaves][4 * (kMaxN + 1)];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar cell indexing
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
    // XCD-contiguous block numbering (blocks are dispatched to the 8 XCDs round robin)
    const long long nb = gridDim.x, b = blockIdx.x;
    const long long xcd = b & 7, q8 = nb >> 3, r8 = nb & 7;
    const long long lb = xcd * q8 + (xcd < r8 ? xcd : r8) + (b >> 3);
    const int gi = find_instance(A.base, A.B, lb);
    const int inst = A.ilist[gi];
    const ChanDesc& I = A.inst[inst];
    const int NL = I.NL, NX = I.NX, NV = I.NV, Q1 = I.Q1, Q2 = I.Q2;
    const double* tab = A.tab + I.offT;

    // ---- the block's instance: momentum-derivative kernels into LDS, zero-padded
    for (int x = threadIdx.x; x < 16 * T1 * 16 * T1; x += kChanWaves * kWave) {
        const int r = x / (16 * T1), c = x - r * (16 * T1);
        const bool ok = r < Q1 && c < Q1;
        k1s[r * S1 + c] = T(ok ? tab[I.tK1 + r * Q1 + c] : 0.0);
        kt1s[r * S1 + c] = T(ok ? tab[I.tKt1 + r * Q1 + c] : 0.0);
    }
    for (int x = threadIdx.x; x < 16 * T2 * 16 * T2; x += kChanWaves * kWave) {
        const int r = x / (16 * T2), c = x - r * (16 * T2);
        const bool ok = r < Q2 && c < Q2;
        k2s[r * S2 + c] = T(ok ? tab[I.tK2 + r * Q2 + c] : 0.0);
        kt2s[r * S2 + c] = T(ok ? tab[I.tKt2 + r * Q2 + c] : 0.0);
    }
    __syncthreads();   // the only block-wide barrier; the wavefronts are independent below

    const int lbi = (int)(lb - A.base[gi]);
    const int NLi = NL > 6 ? NL - 6 : 0, NXi = NX > 6 ? NX - 6 : 0;   // interior extent
    int p, s;
    if (!BND) {
        // interior cells in lambda strips of W cells, each swept along xi, kChanWaves
        // consecutive lambda cells per block (the stencil neighbours of a block are then
        // recent blocks of the same XCD)
        const int W = I.strip, bpw = W / kChanWaves;
        const int strip = lbi / (NXi * bpw), rem = lbi - strip * (NXi * bpw);
        p = 3 + rem / bpw;
        s = 3 + strip * W + (rem - (rem / bpw) * bpw) * kChanWaves + wave;
        if (s >= NL - 3) return;
    } else {
        // edge bands: the rows s < 3, s >= NL - 3 across all columns, then the columns
        // p < 3, p >= NX - 3 of the interior rows
        const int rA = NL < 6 ? NL : 6, cA = NX < 6 ? NX : 6;
        const int c = lbi * kChanWaves + wave;
        if (c < rA * NX) {
            const int r = c % rA;
            p = c / rA;
            s = r < 3 ? r : NL - rA + r;
        } else {
            const int c2 = c - rA * NX;
            if (c2 >= NLi * cA) return;
            const int r = c2 % cA;
            p = r < 3 ? r : NX - cA + r;
            s = 3 + c2 / cA;
        }
    }
    const int cell = p * NL + s;
    const T eps = T(I.weno_eps);
    T* tr = trs[wave];
    T* lcb = lcs[wave];
    double* gf = gsh[wave];
    double* ec = ecs[wave];
    const double* Wm = tab + I.tWm;   // moment weights W_k (FP32 path only)

    // ---- lane items: item t = (I T2 + J) 4 + c is node i = 16 I + 4 c + g, j = 16 J + n
    double plv[T1][4], pxv[T2];
#pragma unroll
    for (int I_ = 0; I_ < T1; ++I_)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = 16 * I_ + 4 * c + g;
            plv[I_][c] = i < Q1 ? tab[I.tp1 + i] : 0.0;
        }
#pragma unroll
    for (int J = 0; J < T2; ++J) pxv[J] = 16 * J + n < Q2 ? tab[I.tp2 + 16 * J + n] : 0.0;
    auto item_i = [&](int t) { return 16 * (t / (4 * T2)) + 4 * (t & 3) + g; };
    auto item_j = [&](int t) { return 16 * ((t >> 2) % T2) + n; };
    auto item_ok = [&](int t) { return item_i(t) < Q1 && item_j(t) < Q2; };
    auto item_k = [&](int t) { return item_ok(t) ? item_i(t) * Q2 + item_j(t) : 0; };
    auto item_pl = [&](int t) { return plv[t / (4 * T2)][t & 3]; };
    auto item_px = [&](int t) { return pxv[(t >> 2) % T2]; };

    const T* F = static_cast<const T*>(A.Fin) + I.offF;
    const size_t dstride = (size_t)NX * NL * NV, xstride = (size_t)NL * NV;
    const T* Fcell = F + ((size_t)p * NL + s) * NV;

    // ---- moments of the cell (FP64 wavefront sums)
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
#pragma unroll
    for (int t = 0; t < NI; ++t) {
        if (!item_ok(t)) continue;
        const int k = item_k(t);
        double f0 = (double)Fcell[k], f1 = (double)Fcell[dstride + k];
        if (F32) {
            f0 *= Wm[k];
            f1 *= Wm[k];
        }
        const double a = item_pl(t), c = item_px(t);
        m0 += f0;
        m1 += a * f0;
        m2 += c * f0;
        m3 += (a * a + c * c) * f0;
        m4 += f1;
    }
    const double nd = wave_sum(m0), u1 = wave_sum(m1) / nd, u2 = wave_sum(m2) / nd;
    const double Tc = (wave_sum(m3) + wave_sum(m4) - nd * (u1 * u1 + u2 * u2)) / (3.0 * nd);
    const double itau = 1.0 / tau_of(I.tau_model, I.Kn, nd, Tc);

    // ---- equilibrium factors g1(p^lambda_i), g2(p^xi_j) of the cell (LDS, this wavefront)
    // lane 2 a + sg: axis a, side sg (a half-range axis has two coefficient sets)
    if (lane < 4) {
        const int ax = lane >> 1, sg = lane & 1, kind = ax ? I.kind2 : I.kind1, N = ax ? I.N2 : I.N1;
        if (kind == 1 || sg == 0)
            axis_coef_side(kind, N, ax ? u2 : u1, Tc, tab + (ax ? I.tC2 : I.tC1), tab + (ax ? I.tisf2 : I.tisf1), sg,
                           ec + ax * 2 * (kMaxN + 1) + sg * (N + 1));
    }
    wave_lds_fence();
    if (lane < Q1 + Q2) {
        const bool ax1 = lane < Q1;
        const int node = ax1 ? lane : lane - Q1;
        const int nbas = ax1 ? I.N1 + 1 : I.N2 + 1;
        const double* brow = tab + (ax1 ? I.tB1 : I.tB2) + node * nbas;
        const double* co = ec + (ax1 ? 0 : 2 * (kMaxN + 1)) +
                           (((ax1 ? I.kind1 : I.kind2) == 1 && node >= (ax1 ? I.Qh1 : I.Qh2)) ? nbas : 0);
        // all entries read at once (indices kept in bounds), the terms past nbas dropped by
        // a select: five independent loads instead of a chain of dependent ones
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l <= kMaxN; ++l) {
            const double t = fma(brow[l < nbas ? l : nbas - 1], co[l], acc);
            acc = l < nbas ? t : acc;
        }
        gf[lane] = acc;
    }

    // ---- wall densities of this xi column (lambda = -1: emitted p^lambda > 0; +1: < 0),
    // FP64 sums of the wall-bound flux
    double nw_lo = 0.0, nw_hi = 0.0;
    if (BND && s < 3 && !I.half) {
        double w = 0.0;
        const T* C0 = F + (size_t)p * NL * NV;
#pragma unroll
        for (int t = 0; t < NI; ++t)
            if (item_ok(t) && item_pl(t) < 0) {
                const int k = item_k(t);
                const T F1 = C0[k], F2 = C0[NV + k], F3 = C0[2 * NV + k];
                const T g0 = T(3) * F1 - T(3) * F2 + F3, gm1 = T(6) * F1 - T(8) * F2 + T(3) * F3;
                const double fl = (double)weno5<T>(F3, F2, F1, g0, gm1, eps);
                w += item_pl(t) * (F32 ? Wm[k] * fl : fl);
            }
        nw_lo = -wave_sum(w) / I.den_lo;
    }
    if (BND && s >= NL - 3) {
        double w = 0.0;
        const T* C0 = F + ((size_t)p * NL + NL - 1) * NV;
#pragma unroll
        for (int t = 0; t < NI; ++t)
            if (item_ok(t) && item_pl(t) > 0) {
                const int k = item_k(t);
                const T G1 = C0[k], G2 = C0[k - NV], G3 = C0[k - 2 * NV];
                const T g0 = T(3) * G1 - T(3) * G2 + G3, gp1 = T(6) * G1 - T(8) * G2 + T(3) * G3;
                const double fl = (double)weno5<T>(G3, G2, G1, g0, gp1, eps);
                w += item_pl(t) * (F32 ? Wm[k] * fl : fl);
            }
        nw_hi = -wave_sum(w) / I.den_hi;
    }

    // ---- flow-rate ends (Sec. VI.C.1-2): the density of the row's entering Maxwellian that
    // makes the row's flow rate sum_k p^y F_face the prescribed one, from FP64 sums of the
    // leaving populations of the end cell (p^y = V^xi / (1 + phi) at the end face)
    double nin_row = 0.0, nout_row = 0.0;
    if (BND && I.ends == 1 && (p < 3 || p >= NX - 3)) {
        const bool at_in = p < 3;
        const int f = at_in ? 0 : NX;
        const double cf = tab[I.txc + (size_t)f * NL + s], af = tab[I.txa + (size_t)f * NL + s];
        const double ipf = at_in ? I.ipf_in : I.ipf_out;
        const T* C0 = F + ((size_t)(at_in ? 0 : NX - 1) * NL + s) * NV;
        double w = 0.0;
#pragma unroll
        for (int t = 0; t < NI; ++t)
            if (item_ok(t)) {
                const int k = item_k(t);
                const double py = cf * (item_px(t) - af * item_pl(t)) * ipf;
                if (at_in ? py <= 0.0 : py >= 0.0) {
                    const double fv = (double)C0[k];
                    w += py * (F32 ? Wm[k] * fv : fv);
                }
            }
        w = wave_sum(w);
        const double nr = (tab[I.tQrow + (at_in ? 0 : NL) + s] - w) / tab[I.tden + (at_in ? 0 : NL) + s];
        if (at_in) nin_row = nr;
        else nout_row = nr;
    }

    // ---- per-cell geometry
    const T glxx = T(tab[I.tglxx + cell]), gxll = T(-tab[I.tglxl + cell]);
    const T al = T(tab[I.tal + cell]), ar = T(tab[I.tar + cell]);
    const T idl = T(1.0 / tab[I.tdlam + s]), idx = T(1.0 / tab[I.tdchi + p]);
    const double* xc = tab + I.txc;
    const double* xa = tab + I.txa;
    const T xc0 = T(xc[(size_t)p * NL + s]), xa0 = T(xa[(size_t)p * NL + s]);
    const T xc1 = T(xc[(size_t)(p + 1) * NL + s]), xa1 = T(xa[(size_t)(p + 1) * NL + s]);
    const T xcin = T(xc[s]), xain = T(xa[s]), xcout = T(xc[(size_t)NX * NL + s]),
            xaout = T(xa[(size_t)NX * NL + s]);
    const bool lam_interior = !BND || (s >= 3 && s < NL - 3), xi_interior = !BND || (p >= 3 && p < NX - 3);
    const bool lonly = A.l_only != 0;
    const double dt = lonly ? 1.0 : I.dt;
    const T ca = T(A.ca), cb = T(A.cb), ccdt = T(A.cc * dt);
    const T Tcell = T(Tc), itauT = T(itau);
    const double* iW = tab + I.tiW;
    wave_lds_fence();
    // The FP32 interior variant of one-tile velocity sets keeps the cell's F and the
    // equilibrium factors in registers through the advection loop; the others, at their
    // register limit, read both back from LDS in the BGK step (held in registers they were
    // spilled to scratch memory; the two-tile FP32 interior variant reads them back to run
    // 4 wavefronts per SIMD instead of 3: 64-channel batch 7.09 -> 7.61 G/s; its edge-band
    // variant runs 3 instead of 2, 7.61 -> 7.78 G/s).
    constexpr bool kRegs = F32 && !BND && T1 * T2 == 1;
    T g1v[T1][4], g2v[T2];
    if (kRegs) {
#pragma unroll
        for (int I_ = 0; I_ < T1; ++I_)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                g1v[I_][c] = T(16 * I_ + 4 * c + g < Q1 ? nd * gf[16 * I_ + 4 * c + g] : 0.0);
#pragma unroll
        for (int J = 0; J < T2; ++J) g2v[J] = T(16 * J + n < Q2 ? gf[Q1 + 16 * J + n] : 0.0);
    }

#pragma unroll 1
    for (int d = 0; d < 2; ++d) {
        const T* Fd = Fcell + d * dstride;
        const double* fw = tab + I.tfw + d * NV;
        T fc[NI];
#pragma unroll
        for (int t = 0; t < NI; ++t) fc[t] = item_ok(t) ? Fd[item_k(t)] : T(0);

        // momentum derivatives (Sec. IV.C) as 16x16x4 MFMA products:
        //   d/dp^lambda: K1 F, Kt1 F (F in its own registers);
        //   d/dp^xi:     F K2^T, F Kt2^T (F from the transpose buffer)
#pragma unroll
        for (int t = 0; t < NI; ++t) tr[item_i(t) * RS + item_j(t)] = fc[t];
        wave_lds_fence();
#pragma unroll
        for (int I_ = 0; I_ < T1; ++I_)
#pragma unroll
            for (int J = 0; J < T2; ++J) {
                acc_t k1 = {0, 0, 0, 0}, kt1 = {0, 0, 0, 0}, k2 = {0, 0, 0, 0}, kt2 = {0, 0, 0, 0};
                const int prow = 16 * I_ + mfma_row<T>(n);
#pragma unroll
                for (int I2 = 0; I2 < T1; ++I2)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const T bf = fc[(I2 * T2 + J) * 4 + c];
                        const int col = 16 * I2 + 4 * c + g;
                        k1 = Acc4<T>::mfma(k1s[prow * S1 + col], bf, k1);
                        kt1 = Acc4<T>::mfma(kt1s[prow * S1 + col], bf, kt1);
                    }
#pragma unroll
                for (int J2 = 0; J2 < T2; ++J2)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int col = 16 * J2 + 4 * c + g;
                        const T af = tr[prow * RS + col];
                        k2 = Acc4<T>::mfma(af, k2s[(16 * J + n) * S2 + col], k2);
                        kt2 = Acc4<T>::mfma(af, kt2s[(16 * J + n) * S2 + col], kt2);
                    }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int t = (I_ * T2 + J) * 4 + c;
                    const T a = T(item_pl(t)), q = T(item_px(t));
                    lcb[item_i(t) * RS + item_j(t)] =
                        glxx * (q * q * k1[c] - a * kt2[c]) + gxll * (a * a * k2[c] - q * kt1[c]);
                }
            }
        wave_lds_fence();   // the buffer is rewritten for the next distribution

        // advection through the four faces: a rolled loop over the lane's items (their F
        // and L live in this lane's slots of the LDS rows), one item in registers at a time.
        // Cells whose stencils stay inside the grid (most of them) take a loop without the
        // ghost logic, so its conditions and offsets do not occupy registers there.
        // Interior cells address their stencil as one buffer over the columns p-3 .. p+3 from
        // row s: one lane offset and wavefront-uniform offsets per neighbour, so the twelve
        // loads of an item need no 64-bit lane addresses (the span, 7 NL NV values, is checked
        // against the 32-bit buffer range at channel creation).
        const __amdgpu_buffer_rsrc_t rSt = buf_rsrc(BND ? Fd : Fd - 3 * xstride,
                                                    BND ? 0u : 7u * (unsigned)xstride * (unsigned)sizeof(T));
        const unsigned xsb = (unsigned)xstride * (unsigned)sizeof(T), nvb = (unsigned)NV * (unsigned)sizeof(T);
        auto advect = [&](auto interior_tag) {
            constexpr bool interior = decltype(interior_tag)::value;
#pragma unroll 1
            for (int t = 0; t < NI; ++t) {
                const int i = 16 * (t / (4 * T2)) + 4 * (t & 3) + g, j = 16 * ((t >> 2) % T2) + n;
                if (i >= Q1 || j >= Q2) continue;
                const int k = i * Q2 + j;
                const T plt = T(tab[I.tp1 + i]), pxt = T(tab[I.tp2 + j]);
                const T fct = tr[i * RS + j];
                T lw[7], xw[7];
                if constexpr (interior) {
                    const unsigned ko = (unsigned)k * (unsigned)sizeof(T);
#pragma unroll
                    for (int q = 0; q < 7; ++q) {   // (q - 3) nvb wraps: the sum is the true offset
                        lw[q] = q == 3 ? fct : buf_load<T>(rSt, ko, 3u * xsb + (unsigned)(q - 3) * nvb);
                        xw[q] = q == 3 ? fct : buf_load<T>(rSt, ko, (unsigned)q * xsb);
                    }
                } else if (lam_interior) {
#pragma unroll
                    for (int q = 0; q < 7; ++q) lw[q] = q == 3 ? fct : Fd[(q - 3) * NV + k];
                } else {
                    const T* Col = Fd - (size_t)s * NV;   // cell (p, 0)
#pragma unroll
                    for (int q = 0; q < 7; ++q) {
                        const int cc = s - 3 + q;
                        T v;
                        if (cc >= 0 && cc < NL) {
                            v = Col[(size_t)cc * NV + k];
                        } else if (cc < 0) {
                            if (I.half) {
                                // specular centreline (Sec. VI.C.3): cell -1 - cc, p^lambda reversed
                                v = Col[(size_t)(-1 - cc) * NV + ((i + I.Qh1) % Q1) * Q2 + j];
                            } else if (plt > T(0)) {
                                v = T(nw_lo * fw[k]);                                // Eq. weno_populate
                            } else {
                                const T F1 = Col[k], F2 = Col[NV + k], F3 = Col[2 * NV + k];
                                v = cc == -1 ? T(3) * F1 - T(3) * F2 + F3              // Eq. extrapol
                                             : cc == -2 ? T(6) * F1 - T(8) * F2 + T(3) * F3 : T(0);
                            }
                        } else {
                            if (plt < T(0)) {
                                v = T(nw_hi * fw[k]);
                            } else {
                                const T G1 = Col[(size_t)(NL - 1) * NV + k], G2 = Col[(size_t)(NL - 2) * NV + k],
                                        G3 = Col[(size_t)(NL - 3) * NV + k];
                                v = cc == NL ? T(3) * G1 - T(3) * G2 + G3
                                             : cc == NL + 1 ? T(6) * G1 - T(8) * G2 + T(3) * G3 : T(0);
                            }
                        }
                        lw[q] = v;
                    }
                }
                if constexpr (interior) {
                } else if (xi_interior) {
#pragma unroll
                    for (int q = 0; q < 7; ++q)
                        xw[q] = q == 3 ? fct : Fd[(ptrdiff_t)(q - 3) * (ptrdiff_t)xstride + k];
                } else {
                    const T vin = xcin * (pxt - xain * plt), vout = xcout * (pxt - xaout * plt);
                    const T* Row = Fd - (size_t)p * xstride;   // cell (0, s)
#pragma unroll
                    for (int q = 0; q < 7; ++q) {
                        const int cc = p - 3 + q;
                        T v;
                        if (cc >= 0 && cc < NX) {
                            v = Row[(size_t)cc * xstride + k];
                        } else if (cc < 0) {
                            const T ent = I.ends == 1 ? T(nin_row * tab[I.tfrow + ((size_t)s * 2 + d) * NV + k])
                                                      : T(tab[I.tfin + d * NV + k]);
                            v = vin > T(0) ? ent : Row[k];
                        } else {
                            const T ent = I.ends == 1
                                              ? T(nout_row * tab[I.tfrow + ((size_t)(NL + s) * 2 + d) * NV + k])
                                              : T(tab[I.tfout + d * NV + k]);
                            v = vout < T(0) ? ent : Row[(size_t)(NX - 1) * xstride + k];
                        }
                        xw[q] = v;
                    }
                }
                // faces s -+ 1/2 between window cells 2|3 and 3|4, upwinded by the sign of
                // p^lambda; faces p -+ 1/2 likewise by the sign of V^xi on each face (one face
                // at a time: the four WENO chains are kept from being interleaved, which would
                // raise the register demand)
                const bool pos = plt > T(0);
                const T Fl = weno_face<T>(pos, lw[0], lw[1], lw[2], lw[3], lw[4], lw[5], eps);
                T adv_l = -al * Fl;
                __builtin_amdgcn_sched_barrier(0);
                const T Fr = weno_face<T>(pos, lw[1], lw[2], lw[3], lw[4], lw[5], lw[6], eps);
                adv_l += ar * Fr;
                __builtin_amdgcn_sched_barrier(0);
                const T V0 = xc0 * (pxt - xa0 * plt), V1 = xc1 * (pxt - xa1 * plt);
                const T X0 = weno_face<T>(V0 > T(0), xw[0], xw[1], xw[2], xw[3], xw[4], xw[5], eps);
                T adv_x = -V0 * X0;
                __builtin_amdgcn_sched_barrier(0);
                const T X1 = weno_face<T>(V1 > T(0), xw[1], xw[2], xw[3], xw[4], xw[5], xw[6], eps);
                adv_x += V1 * X1;
                lcb[i * RS + j] -= plt * adv_l * idl + adv_x * idx;
            }
        };
        if (!BND) advect(std::true_type{});
        else advect(std::false_type{});

        // BGK, RK combination, store, residual partials (FP64).  The variants at their
        // register limit address F_n, the output and the residual weights as buffers of the
        // cell's populations (a wavefront-uniform base and 32-bit lane offsets), so that no
        // 64-bit lane addresses stay live across the loop.
        const size_t cofs = I.offF + d * dstride + ((size_t)p * NL + s) * NV;
        const T* Fn = A.Fn ? static_cast<const T*>(A.Fn) + cofs : nullptr;
        T* Fo = static_cast<T*>(A.Fout) + cofs;
        const __amdgpu_buffer_rsrc_t rFn = buf_rsrc(Fn, Fn ? NV * (unsigned)sizeof(T) : 0u);
        const __amdgpu_buffer_rsrc_t rFo = buf_rsrc(Fo, NV * (unsigned)sizeof(T));
        const __amdgpu_buffer_rsrc_t rW = buf_rsrc(iW, NV * (unsigned)sizeof(double));
        double rd = 0.0, rn = 0.0;
#pragma unroll
        for (int t = 0; t < NI; ++t) {
            if (!item_ok(t)) continue;
            const int k = item_k(t);
            T fe = kRegs ? g1v[t / (4 * T2)][t & 3] * g2v[(t >> 2) % T2]
                         : T(nd * gf[item_i(t)]) * T(gf[Q1 + item_j(t)]);
            if (d) fe *= Tcell;
            const T fct = kRegs ? fc[t] : tr[item_i(t) * RS + item_j(t)];
            const T L = lcb[item_i(t) * RS + item_j(t)] - (fct - fe) * itauT;
            T out;
            if (lonly) {
                out = L;
            } else {
                const T fn = ca == T(0) ? T(0) : kRegs ? Fn[k] : buf_load<T>(rFn, (unsigned)k * (unsigned)sizeof(T));
                out = ca * fn + cb * fct + ccdt * L;
                const double iw = kRegs ? iW[k] : buf_load<double>(rW, (unsigned)k * 8u), dd = (double)out - (double)fn;
                rd += dd * dd * iw;
                rn += (double)fn * (double)fn * iw;
            }
            if (kRegs) Fo[k] = out;
            else buf_store(rFo, (unsigned)k * (unsigned)sizeof(T), 0u, out);
        }
        if (A.rpart) {
            rd = wave_sum(rd);
            rn = wave_sum(rn);
            if (lane == 0) {
                const double vol = tab[I.tvol + cell];
                A.rpart[((size_t)(I.offC + cell) * 2 + d) * 2] = vol * rd;
                A.rpart[((size_t)(I.offC + cell) * 2 + d) * 2 + 1] = vol * rn;
            }
        }
    }
}

// Rest state of every instance: the wall Maxwellian f_eq(1, 0, T_w) in every cell (FP64;
// grid-stride over the populations, since a batch may hold more than 2^32 of them while
// one dispatch covers fewer work-items).
__global__ __launch_bounds__(256) void channel_rest(const ChanDesc* insts, const long long* sbase, int B,
                                                    const double* tab_all, double* F64) {
    const long long total = sbase[B], stride = (long long)gridDim.x * 256;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += stride) {
        const int inst = find_instance(sbase, B, e);
        const ChanDesc& I = insts[inst];
        const long long loc = e - sbase[inst];
        const int k = (int)(loc % I.NV);
        const int d = loc >= (long long)I.NX * I.NL * I.NV ? 1 : 0;
        F64[(size_t)I.offF + (size_t)loc] = tab_all[I.offT + I.tfw + d * I.NV + k];
    }
}

// FP64 state <-> FP32 state scaled by 1/W_k (grid-stride over the populations).
template <bool TO32>
__global__ __launch_bounds__(256) void channel_convert(const ChanDesc* insts, const long long* sbase, int B,
                                                       const double* tab_all, double* F64, float* F32) {
    const long long total = sbase[B], stride = (long long)gridDim.x * 256;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += stride) {
        const int inst = find_instance(sbase, B, e);
        const ChanDesc& I = insts[inst];
        const long long loc = e - sbase[inst];
        const int k = (int)(loc % I.NV);
        const double w = tab_all[I.offT + I.tWm + k];
        const size_t x = (size_t)I.offF + (size_t)loc;
        if (TO32) F32[x] = (float)(F64[x] / w);
        else F64[x] = (double)F32[x] * w;
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
__global__ __launch_bounds__(kMaxNV) void channel_diag(const ChanDesc* insts, const long long* cbase, int B,
                                                             const double* tab_all, const double* F, double* diag) {
    __shared__ double sh[16 * 5];
    for (long long b = blockIdx.x; b < cbase[B]; b += gridDim.x) {   // uniform per block
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
}

// ---------------------------------------------------------------- flow diagnostics
// Cartesian velocity of cell (p, s) from its triad components (Eq. canalie_u): the triad
// of the cell is the Cartesian frame turned by the angle whose tangent is a = lambda phi'.
__device__ __forceinline__ void cart_velocity(const double* dg, const double* lamc, const double* dphi, int NL, int p,
                                              int s, double& ux, double& uy) {
    const double* m = dg + ((size_t)p * NL + s) * 5;
    if (dphi == nullptr) {   // Cartesian-split instance: the moments are Cartesian already
        ux = m[1];
        uy = m[2];
        return;
    }
    const double a = lamc[s] * dphi[p], c = 1.0 / sqrt(1.0 + a * a);
    ux = (m[1] + a * m[2]) * c;
    uy = (m[2] - a * m[1]) * c;
}

// Derivative at xt of the quadratic through (x0, x1, x2): weights of the three samples
// (derivatives of the Lagrange basis polynomials at xt).
__device__ __forceinline__ void quad_deriv_weights(double xt, double x0, double x1, double x2, double* w) {
    w[0] = ((xt - x1) + (xt - x2)) / ((x0 - x1) * (x0 - x2));
    w[1] = ((xt - x0) + (xt - x2)) / ((x1 - x0) * (x1 - x2));
    w[2] = ((xt - x0) + (xt - x1)) / ((x2 - x0) * (x2 - x1));
}

// First of the three nodes that differentiate at node i of n (n >= 3): the neighbours
// inside, one-sided at the ends (Sec. VI.F).
__device__ __forceinline__ int quad_first(int i, int n) { return i == 0 ? 0 : (i == n - 1 ? n - 3 : i - 1); }

// Flow diagnostics of one instance (Sec. VI.D, VI.F), one thread per xi column p, from
// the cell moments diag (n, u^lambda, u^xi, T, content): Cartesian velocity, P = n T,
// vorticity (Eq. canalie_vorti, three-point derivatives on the cell centres), the stream
// function on the lambda faces (d psi = -n u^y (1 + phi) d lambda, zero at lambda = 0)
// and the pressure extrapolated linearly to the faces 0 and NL.
__global__ __launch_bounds__(64) void channel_fields(const ChanDesc* inst, const double* tab_all, const double* diag,
                                                     double* out) {
    const ChanDesc& D = *inst;
    const int NL = D.NL, NX = D.NX;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NX) return;
    const double* geo = tab_all + D.offT + D.tgeo;
    const double *phi = geo, *xic = geo + 2 * NX, *lamf = geo + 3 * NX, *lamc = lamf + NL + 1;
    const double* dphi = D.cartesian ? nullptr : geo + NX;
    const double* dg = diag + (size_t)D.offC * 5;
    const size_t nc = (size_t)NX * NL;
    double *oux = out, *ouy = out + nc, *oP = out + 2 * nc, *oom = out + 3 * nc, *opsi = out + 4 * nc + (size_t)p * (NL + 1),
           *oPw = out + 4 * nc + (size_t)NX * (NL + 1);
    const double opf = 1.0 + phi[p];
    const int q0 = quad_first(p, NX);
    double wx[3];
    quad_deriv_weights(xic[p], xic[q0], xic[q0 + 1], xic[q0 + 2], wx);
    double cum = 0.0;
    opsi[0] = 0.0;
    for (int s = 0; s < NL; ++s) {
        const size_t ci = (size_t)p * NL + s;
        const double n = dg[ci * 5], T = dg[ci * 5 + 3];
        double ux, uy;
        cart_velocity(dg, lamc, dphi, NL, p, s, ux, uy);
        oux[ci] = ux;
        ouy[ci] = uy;
        oP[ci] = n * T;
        double dxi = 0.0, dlx = 0.0, dly = 0.0, wl[3];
        const int r0 = quad_first(s, NL);
        quad_deriv_weights(lamc[s], lamc[r0], lamc[r0 + 1], lamc[r0 + 2], wl);
        for (int e = 0; e < 3; ++e) {
            double vx, vy;
            cart_velocity(dg, lamc, dphi, NL, q0 + e, s, vx, vy);
            dxi += wx[e] * vx;
            cart_velocity(dg, lamc, dphi, NL, p, r0 + e, vx, vy);
            dlx += wl[e] * vx;
            dly += wl[e] * vy;
        }
        const double aa = lamc[s] * geo[NX + p];   // lambda phi'
        oom[ci] = -dxi + (dly + aa * dlx) / opf;
        cum += n * uy * (opf * (lamf[s + 1] - lamf[s]));
        opsi[s + 1] = cum;
    }
    // lambda = 0 is face NL / 2 of the full width (the middle of cell (NL - 1) / 2 for odd
    // NL) and face 0 of the half channel
    const int s0 = D.half ? 0 : NL / 2;
    const double fr = (D.half || NL % 2 == 0) ? 0.0 : 0.5;
    const double ref = (1.0 - fr) * opsi[s0] + fr * opsi[s0 + 1];
    for (int s = 0; s <= NL; ++s) opsi[s] = ref - opsi[s];
    for (int side = 0; side < 2; ++side) {
        const int e = side ? NL : 0, i1 = side ? NL - 1 : 0, i2 = side ? NL - 2 : 1;
        const size_t c1 = (size_t)p * NL + i1, c2 = (size_t)p * NL + i2;
        const double P1 = dg[c1 * 5] * dg[c1 * 5 + 3], P2 = dg[c2 * 5] * dg[c2 * 5 + 3];
        const double lw = lamf[e], l1 = lamc[i1], l2 = lamc[i2];
        oPw[(size_t)side * NX + p] = ((lw - l2) * P1 - (lw - l1) * P2) / (l1 - l2);
    }
}

// ---------------------------------------------------------------- population kernel
// Channel stage with a block per cell and a thread per velocity (FP64), for both momentum
// forms.  The block sums its cell's moments itself, builds the equilibrium factors in
// LDS, finds n_w of the column's walls and the flow-rate densities of its row when its
// stencil reaches them, then per population: the four WENO faces with wall, centreline
// and end ghosts, the flux difference, the force (vielbein form), BGK, the RK combine.
//   vielbein (Sec. VI.A-C): V^lambda = (face factor) p^lambda from the per-cell tables,
//     V^xi = c_f (p^xi - a_f p^lambda) at the xi faces, the four projected derivatives
//     Gamma_lxx [(p^xi)^2 K1 F - p^lambda Kt2 F] - Gamma_lxl [(p^lambda)^2 K2 F - p^xi Kt1 F]
//     as dot products over the cell's populations staged in LDS -- the form for velocity
//     sets too sparse for the 16 x 16 tiles of channel_stage (e.g. 5 p^xi nodes);
//   Cartesian split (Sec. VI.G, Eq. canalie_coord_beq_cons): axes p^x / p^y, no force,
//     V^lambda = (p^x - lambda a_p p^y) / (1 + phi_p) with the discrete metric
//     a_p = (1 + phi_p)(phi_{p+1/2} - phi_{p-1/2}) / dchi_p (free-stream preserving),
//     V^xi = (1 + phi) p^y; walls by the sign of V^lambda at the wall face
//     (Eq. canalie_coord_nw); flow-rate ends with the Cartesian profile velocity (0, Q_s).
// A population is wall-bound or emitted by the sign of V^lambda at the wall face (for the
// vielbein form the sign of p^lambda; the positive face factor cancels in n_w).  The half
// channel mirrors the ax1 momentum at the centreline.  Each thread takes the velocities
// k = threadIdx.x + j kPopThreads.
constexpr int kPopThreads = 256;
template <bool CART>   // the momentum form of every listed instance
__global__ __launch_bounds__(kPopThreads) void pop_stage(ChanArgs A) {
    __shared__ double sh[16 * 5];
    __shared__ double ec[4 * (kMaxN + 1)];
    __shared__ double gq[4 * kMaxQ];   // g(p) of the nodes of both axes
    __shared__ double fl[2 * kMaxNV];  // the cell's populations (vielbein force contractions)
    const long long b = blockIdx.x;
    const int gi = find_instance(A.base, A.B, b);
    const ChanDesc& I = A.inst[A.ilist[gi]];
    const int cell = (int)(b - A.base[gi]);
    const int NL = I.NL, NX = I.NX, NV = I.NV, Q1 = I.Q1, Q2 = I.Q2, N1 = I.N1, N2 = I.N2;
    const int p = cell / NL, s = cell - p * NL;
    const double* tab = A.tab + I.offT;
    const double* F = static_cast<const double*>(A.Fin) + I.offF;
    const size_t dsz = (size_t)NX * NL * NV;
    auto at = [&](int d, int pp, int ss, int k) -> double { return F[d * dsz + ((size_t)pp * NL + ss) * NV + k]; };
    auto pxk = [&](int k) -> double { return tab[I.tp1 + k / Q2]; };
    auto pyk = [&](int k) -> double { return tab[I.tp2 + k % Q2]; };

    // moments of the cell (Sec. IV.A) and the relaxation time
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < NV; k += kPopThreads) {
        const double px = pxk(k), py = pyk(k), f0 = at(0, p, s, k);
        m[0] += f0;
        m[1] += px * f0;
        m[2] += py * f0;
        m[3] += (px * px + py * py) * f0;
        m[4] += at(1, p, s, k);
    }
    block_sums<5>(m, sh);
    const double n = m[0], ux = m[1] / n, uy = m[2] / n;
    const double T = (m[3] + m[4] - n * (ux * ux + uy * uy)) / (3.0 * n);
    const double itau = 1.0 / tau_of(I.tau_model, I.Kn, n, T);
    // equilibrium coefficients (Sec. IV.D): thread 2 ax + sg, both sides of both axes
    if (threadIdx.x < 4) {
        const int ax = threadIdx.x >> 1, sg = threadIdx.x & 1, N = ax ? N2 : N1;
        axis_coef_side(ax ? I.kind2 : I.kind1, N, ax ? uy : ux, T, tab + (ax ? I.tC2 : I.tC1),
                       tab + (ax ? I.tisf2 : I.tisf1), sg, ec + ax * 2 * (kMaxN + 1) + sg * (N + 1));
    }
    constexpr bool cart = CART;
    if (!cart)
        for (int x = threadIdx.x; x < 2 * NV; x += kPopThreads) fl[x] = at(x >= NV, p, s, x >= NV ? x - NV : x);
    __syncthreads();
    for (int t = threadIdx.x; t < Q1 + Q2; t += kPopThreads) {
        const bool ax1 = t < Q1;
        const int node = ax1 ? t : t - Q1, N = ax1 ? N1 : N2;
        const bool minus = ax1 ? (I.kind1 == 1 && node >= I.Qh1) : (I.kind2 == 1 && node >= I.Qh2);
        const double* co = ec + (ax1 ? 0 : 2 * (kMaxN + 1)) + (minus ? N + 1 : 0);
        const double* brow = tab + (ax1 ? I.tB1 : I.tB2) + node * (N + 1);
        double g = 0.0;
        for (int l = 0; l <= N; ++l) g += brow[l] * co[l];
        gq[t] = g;
    }
    __syncthreads();

    // geometry of the column
    const double* geo = tab + I.tgeo;
    const double inv_opf = 1.0 / (1.0 + geo[p]);
    const double* lamf = geo + 3 * NX;
    const double am = cart ? tab[I.tclb + p] : 0.0;
    const double* phif = tab + I.tclb + NX;
    const double* xc = tab + I.txc;   // vielbein: V^xi = xc (p^xi - xa p^lambda) at [xi face][row]
    const double* xa = tab + I.txa;
    // V^lambda at the walls (vielbein: p^lambda, whose positive face factor cancels in n_w)
    auto vwall = [&](double px, double py, bool upper) -> double {
        return cart ? (px + (upper ? -am : am) * py) * inv_opf : px;
    };
    // V^xi at xi face f of this row
    auto vxi = [&](double px, double py, int f) -> double {
        return cart ? (1.0 + phif[f]) * py : xc[(size_t)f * NL + s] * (py - xa[(size_t)f * NL + s] * px);
    };
    const double* fw = tab + I.tfw;
    const double weps = I.weno_eps;
    // n_w of the walls this cell's stencil reaches (Eq. canalie_coord_nw; f' only)
    double nw_lo = 0.0, nw_hi = 0.0;
    if (s < 3 || s >= NL - 3) {
        double w[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = threadIdx.x; k < NV; k += kPopThreads) {
            const double px = pxk(k), py = pyk(k);
            const double vlo = vwall(px, py, false), vhi = vwall(px, py, true);   // at lambda = -1, +1
            if (I.half) {
                // specular centreline: no lower wall
            } else if (vlo < 0.0) {
                const double F1 = at(0, p, 0, k), F2 = at(0, p, 1, k), F3 = at(0, p, 2, k);
                w[0] += vlo * weno5<double>(F3, F2, F1, 3.0 * F1 - 3.0 * F2 + F3, 6.0 * F1 - 8.0 * F2 + 3.0 * F3, weps);
            } else if (vlo > 0.0) {
                w[1] += vlo * fw[k];
            }
            if (vhi > 0.0) {
                const double G1 = at(0, p, NL - 1, k), G2 = at(0, p, NL - 2, k), G3 = at(0, p, NL - 3, k);
                w[2] += vhi * weno5<double>(G3, G2, G1, 3.0 * G1 - 3.0 * G2 + G3, 6.0 * G1 - 8.0 * G2 + 3.0 * G3, weps);
            } else if (vhi < 0.0) {
                w[3] += vhi * fw[k];
            }
        }
        block_sums<4>(w, sh);
        nw_lo = I.half ? 0.0 : -w[0] / w[1];
        nw_hi = -w[2] / w[3];
    }
    // flow-rate ends (Sec. VI.C.1-2): densities of the entering ghosts of this row
    double n_in = 0.0, n_out = 0.0;
    if (I.ends == 1 && (p < 3 || p >= NX - 3)) {
        double w[2] = {0.0, 0.0};
        for (int k = threadIdx.x; k < NV; k += kPopThreads) {
            const double px = pxk(k), py = pyk(k);
            const double vin = vxi(px, py, 0), vout = vxi(px, py, NX);
            // leaving populations carry p^y = V^xi / (1 + phi) through the end faces
            if (vin <= 0.0) w[0] += at(0, 0, s, k) * (vin * I.ipf_in);
            if (vout >= 0.0) w[1] += at(0, NX - 1, s, k) * (vout * I.ipf_out);
        }
        block_sums<2>(w, sh);
        n_in = (tab[I.tQrow + s] - w[0]) / tab[I.tden + s];
        n_out = (tab[I.tQrow + NL + s] - w[1]) / tab[I.tden + NL + s];
    }

    double rp[4] = {0.0, 0.0, 0.0, 0.0};
    const double dt = A.l_only ? 1.0 : I.dt;
    const double dlam = tab[I.tdlam + s], dchi = tab[I.tdchi + p];
    const double* fin = tab + I.tfin;
    const double* fout = tab + I.tfout;
    const double* frow = tab + I.tfrow;
    for (int k = threadIdx.x; k < NV; k += kPopThreads) {
        const int vi = k / Q2, vj = k - vi * Q2;
        const int km = ((vi + I.Qh1) % Q1) * Q2 + vj;   // the p^x-mirrored velocity (half channel)
        const double px = tab[I.tp1 + vi], py = tab[I.tp2 + vj];
        const double vlo = vwall(px, py, false), vhi = vwall(px, py, true);
        const double vl = cart ? (px - lamf[s] * am * py) * inv_opf : tab[I.tal + cell] * px;
        const double vr = cart ? (px - lamf[s + 1] * am * py) * inv_opf : tab[I.tar + cell] * px;
        const double ul = vxi(px, py, p), ur = vxi(px, py, p + 1);
        const double vin = vxi(px, py, 0), vout = vxi(px, py, NX);   // end faces of this row
        const double fe1 = n * gq[vi] * gq[Q1 + vj];
        for (int d = 0; d < 2; ++d) {
            // column values with wall ghosts, row values with reservoir / flow-rate ghosts
            auto colv = [&](int c) -> double {
                if (c >= 0 && c < NL) return at(d, p, c, k);
                if (c < 0 && I.half) return at(d, p, -1 - c, km);
                if (c < 0) {
                    if (vlo > 0.0) return nw_lo * fw[d * NV + k];
                    const double F1 = at(d, p, 0, k), F2 = at(d, p, 1, k), F3 = at(d, p, 2, k);
                    if (c == -1) return 3.0 * F1 - 3.0 * F2 + F3;
                    if (c == -2) return 6.0 * F1 - 8.0 * F2 + 3.0 * F3;
                    return 10.0 * F1 - 15.0 * F2 + 6.0 * F3;
                }
                if (vhi < 0.0) return nw_hi * fw[d * NV + k];
                const double G1 = at(d, p, NL - 1, k), G2 = at(d, p, NL - 2, k), G3 = at(d, p, NL - 3, k);
                if (c == NL) return 3.0 * G1 - 3.0 * G2 + G3;
                if (c == NL + 1) return 6.0 * G1 - 8.0 * G2 + 3.0 * G3;
                return 10.0 * G1 - 15.0 * G2 + 6.0 * G3;
            };
            auto rowv = [&](int c) -> double {
                if (c >= 0 && c < NX) return at(d, c, s, k);
                if (c < 0) {
                    if (vin <= 0.0) return at(d, 0, s, k);
                    return I.ends == 1 ? n_in * frow[((size_t)s * 2 + d) * NV + k] : fin[d * NV + k];
                }
                if (vout >= 0.0) return at(d, NX - 1, s, k);
                return I.ends == 1 ? n_out * frow[((size_t)(NL + s) * 2 + d) * NV + k] : fout[d * NV + k];
            };
            // the two directions one after the other (seven stencil values live at a time)
            double w[7];
            for (int q = 0; q < 7; ++q) w[q] = colv(s - 3 + q);
            const double fc = w[3];
            double adv = (vr * weno_face<double>(vr > 0.0, w[1], w[2], w[3], w[4], w[5], w[6], weps) -
                          vl * weno_face<double>(vl > 0.0, w[0], w[1], w[2], w[3], w[4], w[5], weps)) / dlam;
            for (int q = 0; q < 7; ++q) w[q] = rowv(p - 3 + q);
            adv += (ur * weno_face<double>(ur > 0.0, w[1], w[2], w[3], w[4], w[5], w[6], weps) -
                    ul * weno_face<double>(ul > 0.0, w[0], w[1], w[2], w[3], w[4], w[5], weps)) / dchi;
            double force = 0.0;
            if (!cart) {   // projected momentum derivatives of the two connection terms
                const double* Fd = fl + d * NV;
                const double* K1 = tab + I.tK1 + (size_t)vi * Q1;
                const double* Kt1 = tab + I.tKt1 + (size_t)vi * Q1;
                const double* K2 = tab + I.tK2 + (size_t)vj * Q2;
                const double* Kt2 = tab + I.tKt2 + (size_t)vj * Q2;
                double k1 = 0.0, kt1 = 0.0, k2 = 0.0, kt2 = 0.0;
                for (int ip = 0; ip < Q1; ++ip) {
                    const double f = Fd[ip * Q2 + vj];
                    k1 += K1[ip] * f;
                    kt1 += Kt1[ip] * f;
                }
                for (int jp = 0; jp < Q2; ++jp) {
                    const double f = Fd[vi * Q2 + jp];
                    k2 += K2[jp] * f;
                    kt2 += Kt2[jp] * f;
                }
                force = tab[I.tglxx + cell] * (py * py * k1 - px * kt2) - tab[I.tglxl + cell] * (px * px * k2 - py * kt1);
            }
            const double fe = d ? T * fe1 : fe1;
            const double L = -adv + force - (fc - fe) * itau;
            const size_t o = d * dsz + (size_t)cell * NV + k;
            double out;
            if (A.l_only) {
                out = L;
            } else {
                const double fn = A.ca != 0.0 ? static_cast<const double*>(A.Fn)[I.offF + o] : 0.0;
                out = A.ca * fn + A.cb * fc + A.cc * dt * L;
                const double iw = tab[I.tiW + k], dd = out - fn;
                rp[2 * d] += dd * dd * iw;
                rp[2 * d + 1] += fn * fn * iw;
            }
            static_cast<double*>(A.Fout)[I.offF + o] = out;
        }
    }
    if (A.rpart) {
        block_sums<4>(rp, sh);
        if (threadIdx.x == 0) {
            const double vol = tab[I.tvol + cell];
            for (int d = 0; d < 2; ++d) {
                A.rpart[((size_t)(I.offC + cell) * 2 + d) * 2] = vol * rp[2 * d];
                A.rpart[((size_t)(I.offC + cell) * 2 + d) * 2 + 1] = vol * rp[2 * d + 1];
            }
        }
    }
}

hipError_t launch_channel_stage(int fp32, int T1, int T2, int bnd, long long nblocks, hipStream_t st,
                                const ChanArgs& A) {
    if (nblocks == 0) return hipSuccess;
    const dim3 grid((unsigned)nblocks), block(kChanWaves * kWave);
#define VLB_CHAN_LAUNCH(TT, A1, A2)                                                                  \
    do {                                                                                             \
        if (bnd) hipLaunchKernelGGL((channel_stage<TT, A1, A2, true>), grid, block, 0, st, A);        \
        else hipLaunchKernelGGL((channel_stage<TT, A1, A2, false>), grid, block, 0, st, A);           \
    } while (0)
    if (fp32) {
        if (T1 == 1 && T2 == 1) VLB_CHAN_LAUNCH(float, 1, 1);
        else if (T1 == 2 && T2 == 1) VLB_CHAN_LAUNCH(float, 2, 1);
        else if (T1 == 1 && T2 == 2) VLB_CHAN_LAUNCH(float, 1, 2);
        else return hipErrorInvalidValue;
    } else {
        if (T1 == 1 && T2 == 1) VLB_CHAN_LAUNCH(double, 1, 1);
        else if (T1 == 2 && T2 == 1) VLB_CHAN_LAUNCH(double, 2, 1);
        else if (T1 == 1 && T2 == 2) VLB_CHAN_LAUNCH(double, 1, 2);
        else return hipErrorInvalidValue;
    }
#undef VLB_CHAN_LAUNCH
    return hipGetLastError();
}

// grid of the grid-stride kernels: enough blocks to fill the chip, far below 2^32 work-items
static dim3 stride_grid(long long n, long long per_block) {
    const long long want = (n + per_block - 1) / per_block;
    return dim3((unsigned)std::max(1LL, std::min(want, 1LL << 20)));
}

// Local equilibrium of one instance from per-cell fields prof = [4][NX][NL] (n, u^lambda,
// u^xi, T): f' = n g1(p_i) g2(p_j), f'' = T f' with the equilibrium expansion of the stage
// kernel (Sec. IV.D, Eqs. feq_red, eq_gak_H, eq_gak_hh).  One wavefront per cell; every
// lane computes the cell's axis coefficients (no divergence), then the lanes split the
// velocities.
__global__ __launch_bounds__(256) void channel_init_profile(const ChanDesc* inst, const double* tab_all,
                                                            const double* prof, double* F64) {
    const ChanDesc& I = *inst;
    const long long nc = (long long)I.NX * I.NL;
    const long long cell = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (cell >= nc) return;
    const double* tab = tab_all + I.offT;
    const int NV = I.NV, Q2 = I.Q2, N1 = I.N1, N2 = I.N2;
    const double n = prof[cell], u1 = prof[nc + cell], u2 = prof[2 * nc + cell], T_ = prof[3 * nc + cell];
    double c1[2 * (kMaxN + 1)], c2[2 * (kMaxN + 1)];
    axis_coef(I.kind1, N1, u1, T_, tab + I.tC1, tab + I.tisf1, c1, c1 + (N1 + 1));
    axis_coef(I.kind2, N2, u2, T_, tab + I.tC2, tab + I.tisf2, c2, c2 + (N2 + 1));
    double* out = F64 + (size_t)I.offF + (size_t)cell * NV;
    const size_t dsz = (size_t)nc * NV;
    for (int k = lane; k < NV; k += 64) {
        const int i = k / Q2, j = k - i * Q2;
        const double* e1 = c1 + ((I.kind1 == 1 && i >= I.Qh1) ? N1 + 1 : 0);
        const double* e2 = c2 + ((I.kind2 == 1 && j >= I.Qh2) ? N2 + 1 : 0);
        double g1 = 0.0, g2 = 0.0;
        for (int l = 0; l <= N1; ++l) g1 += tab[I.tB1 + i * (N1 + 1) + l] * e1[l];
        for (int l = 0; l <= N2; ++l) g2 += tab[I.tB2 + j * (N2 + 1) + l] * e2[l];
        const double v = n * g1 * g2;
        out[k] = v;
        out[dsz + k] = T_ * v;
    }
}

hipError_t launch_channel_init_profile(long long ncells, hipStream_t st, const ChanDesc* inst, const double* tab,
                                       const double* prof, double* F64) {
    hipLaunchKernelGGL(channel_init_profile, dim3((unsigned)((ncells + 3) / 4)), dim3(256), 0, st, inst, tab, prof,
                       F64);
    return hipGetLastError();
}

hipError_t launch_channel_rest(long long nelems, hipStream_t st, const ChanDesc* insts, const long long* sbase, int B,
                               const double* tab, double* F64) {
    const dim3 grid = stride_grid(nelems, 256), block(256);
    hipLaunchKernelGGL(channel_rest, grid, block, 0, st, insts, sbase, B, tab, F64);
    return hipGetLastError();
}

hipError_t launch_channel_convert(int to32, long long nelems, hipStream_t st, const ChanDesc* insts,
                                  const long long* sbase, int B, const double* tab, double* F64, float* F32) {
    const dim3 grid = stride_grid(nelems, 256), block(256);
    if (to32) hipLaunchKernelGGL(channel_convert<true>, grid, block, 0, st, insts, sbase, B, tab, F64, F32);
    else hipLaunchKernelGGL(channel_convert<false>, grid, block, 0, st, insts, sbase, B, tab, F64, F32);
    return hipGetLastError();
}

hipError_t launch_channel_reduce(int ninst, hipStream_t st, const ChanDesc* insts, const double* tab,
                                 const double* rpart, double* resid) {
    hipLaunchKernelGGL(channel_reduce, dim3(ninst), dim3(256), 0, st, insts, tab, rpart, resid);
    return hipGetLastError();
}

hipError_t launch_channel_diag(long long ncells_total, int threads, hipStream_t st, const ChanDesc* insts,
                               const long long* cbase, int B, const double* tab, const double* F, double* diag) {
    hipLaunchKernelGGL(channel_diag, stride_grid(ncells_total, 1), dim3(threads), 0, st, insts, cbase, B, tab, F, diag);
    return hipGetLastError();
}

hipError_t launch_channel_fields(int NX, hipStream_t st, const ChanDesc* inst, const double* tab, const double* diag,
                                 double* out) {
    hipLaunchKernelGGL(channel_fields, dim3((unsigned)((NX + 63) / 64)), dim3(64), 0, st, inst, tab, diag, out);
    return hipGetLastError();
}

hipError_t launch_pop_stage(int cartesian, long long ncells, hipStream_t st, const ChanArgs& A) {
    if (ncells == 0) return hipSuccess;
    if (cartesian) hipLaunchKernelGGL(pop_stage<true>, dim3((unsigned)ncells), dim3(kPopThreads), 0, st, A);
    else hipLaunchKernelGGL(pop_stage<false>, dim3((unsigned)ncells), dim3(kPopThreads), 0, st, A);
    return hipGetLastError();
}

}  // namespace vlb
