// Circular-Couette RK stage for large velocity sets (gfx950, FP64): more than 1024
// velocities per cell or more than 64 nodes on the two axes together -- the ballistic
// regime of Sec. V.E needs HH(4;200) x HH(4;10), 8000 velocities, where the p^R kernel
// K1 alone is 400 x 400.  The stage computes the same L[F] and RK combination as the
// one-block-per-run stage kernel (Sec. III.A Eq. rk3; Sec. V.A Eq. boltz_couette_kom;
// walls of Sec. III.F; WENO-5 of Sec. III.C; equilibrium of Sec. IV.D), in three launches
// per instance, because one cell's velocities no longer fit one block:
//   wide_force_prep  the product blocks form Y = K1 F for every (distribution, cell): the
//                p^R derivative kernel of Sec. IV.C as one FP64 MFMA product over the
//                flattened (distribution, cell, p^phi node) columns (v_mfma_f64_16x16x4f64;
//                a block per 16 rows x 64 columns, each K1 fragment feeding four tiles,
//                the four wavefronts splitting the contraction and adding their partial
//                tiles in wavefront order; ragged tiles zero-padded).  The prep blocks after them
//                take, per cell (first prep block), n, T, 1/tau, the equilibrium
//                coefficients and the geometry from the moment sums of the stage input,
//                and per 256 velocities the FP64 partial sums of the wall-bound WENO flux
//                through both walls (Eq. nw), which every update block adds in chunk
//                order into n_w;
//   wide_update  one thread per population: two WENO faces, the flux difference, the
//                force Gamma [(p^phi)^2 Y - p^R F Kt2^T] (the p^phi contraction from the
//                block's rows of F staged in LDS), BGK, the RK combine, the
//                store, and per-block FP64 partial sums of the output's moments and
//                residual in a fixed order;
//   wide_finish  per (distribution, cell): the partial sums added in chunk order into
//                the moment sums the next stage reads and into the residual partials.
// (Folding the finish into the update through a last-arriving-block counter needs a
// device-scope fence in every block, which writes back and invalidates L2 on this chip:
// it made the step 45 % slower than the extra launch.)
#include <hip/hip_runtime.h>

#include "vlb_device.h"
#include "vlb_internal.h"

namespace vlb {

namespace {

constexpr int kWideThreads = 256;   // threads of the prep, update and finish blocks
constexpr int kWidePart = 8;        // partial sums per update block: m0..m3, rd, rn, pad

// Block-wide sums of NQ values in a fixed order: DPP wavefront sums, then the wavefronts
// in index order; sh holds NQ x (waves per block) doubles.
template <int NQ>
__device__ void block_sums(double* v, double* sh) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();
    if (lane == 0)
        for (int q = 0; q < NQ; ++q) sh[q * nw + wave] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[q * nw + w];
        v[q] = s;
    }
}

// Block-wide sum in a fixed order: DPP wavefront sums, then the wavefronts in index order.
__device__ double block_sum(double v, double* sh) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

}  // namespace

__device__ void wide_prep(const WideArgs& A, int chunk, double* sh) {
    const InstDesc& I = *A.inst;
    const double* tab = A.tab + I.offT;
    const int NR = I.NR, NV = I.NV, Q2 = I.Q2, N1 = I.N1, N2 = I.N2;
    const int t = threadIdx.x;
    for (int s = t; s < (chunk == 0 ? NR : 0); s += kWideThreads) {
        const double* ms = A.msum_in + (size_t)(I.offC + s) * 5;
        const double n = ms[0], u1 = ms[1] / n, u2 = ms[2] / n;
        const double T_ = (ms[3] + ms[4] - n * (u1 * u1 + u2 * u2)) / (3.0 * n);
        double* e = A.eq + (size_t)s * kEqStride;
        e[0] = n;
        e[1] = T_;
        e[2] = 1.0 / tau_of(I.tau_model, I.Kn, n, T_);
        axis_coef(I.kind1, N1, u1, T_, tab + I.tC1, tab + I.tisf1, e + 3, e + 3 + (N1 + 1));
        axis_coef(I.kind2, N2, u2, T_, tab + I.tC2, tab + I.tisf2, e + 3 + 2 * (N1 + 1), e + 3 + 2 * (N1 + 1) + (N2 + 1));
        e[kEqGeo] = tab[I.tRf + s] / tab[I.tdchi + s];
        e[kEqGeo + 1] = tab[I.tRf + s + 1] / tab[I.tdchi + s];
        e[kEqGeo + 2] = tab[I.tdchi + s];
        e[kEqGeo + 3] = tab[I.tGam + s];
    }
    // wall-bound flux of f' through each wall face (Eq. nw), ghosts by Eq. extrapol
    const double* Fp = A.Fin + I.offF;
    const double* Wm = tab + I.tWm;
    const double weps = I.weno_eps;
    double ain = 0.0, aout = 0.0;
    const int k = chunk * kWideThreads + t;
    if (k < NV) {
        const double p1 = tab[I.tp1 + k / Q2];
        // f-tilde form: the wall-bound flux is reconstructed from sqrt(g) f
        const double* sg = tab + I.tsqg;
        const bool ft = I.form == 1;
        if (p1 < 0.0) {
            const double F1 = ft ? sg[0] * Fp[k] : Fp[k], F2 = ft ? sg[1] * Fp[NV + k] : Fp[NV + k],
                         F3 = ft ? sg[2] * Fp[2 * NV + k] : Fp[2 * NV + k];
            const double g0 = 3.0 * F1 - 3.0 * F2 + F3, gm1 = 6.0 * F1 - 8.0 * F2 + 3.0 * F3;
            ain += p1 * Wm[k] * weno5<double>(F3, F2, F1, g0, gm1, weps);
        } else if (p1 > 0.0) {
            double G1 = Fp[(size_t)(NR - 1) * NV + k], G2 = Fp[(size_t)(NR - 2) * NV + k],
                   G3 = Fp[(size_t)(NR - 3) * NV + k];
            if (ft) { G1 *= sg[NR - 1]; G2 *= sg[NR - 2]; G3 *= sg[NR - 3]; }
            const double g0 = 3.0 * G1 - 3.0 * G2 + G3, gp1 = 6.0 * G1 - 8.0 * G2 + 3.0 * G3;
            aout += p1 * Wm[k] * weno5<double>(G3, G2, G1, g0, gp1, weps);
        }
    }
    ain = block_sum(ain, sh);
    aout = block_sum(aout, sh);
    if (t == 0) {
        A.nw[2 * chunk] = ain;
        A.nw[2 * chunk + 1] = aout;
    }
}

// Y = K1 F as one product over the flattened columns c = b n2 + j of all (distribution,
// cell) blocks b: C[i][c] = sum_k K1[i][k] F_b[k][j].  A block owns rows 16 I0 .. 16 I0 + 15
// and kWideCols consecutive columns (kWideCols / 16 MFMA tiles sharing each K1 fragment);
// its four wavefronts split the contraction and add their partial tiles in wavefront order.
constexpr int kWideCols = 64;
__device__ void wide_force(const WideArgs& A, long long tile, double (*part)[kWideCols / 16][4][kWave]) {
    constexpr int NT = kWideCols / 16;
    const InstDesc& I = *A.inst;
    const double* tab = A.tab + I.offT;
    const int n1 = I.Q1, n2 = I.Q2, NV = I.NV;
    const int TI = (n1 + 15) / 16;
    const long long NC = (long long)2 * I.NR * n2;   // flattened columns
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int I0 = (int)(tile % TI);
    const long long c0 = tile / TI * kWideCols;
    // wavefront w contracts over k in [w kq, (w + 1) kq), kq a multiple of 4
    const int kq = (n1 + 15) / 16 * 4, kbeg = wave * kq, kend = min(n1, kbeg + kq);
    const int g = lane >> 4, n = lane & 15;
    const double* K1 = tab + I.tK1;
    const int row = 16 * I0 + n;
    // this lane's column of each tile: (distribution, cell) block and p^phi node
    const double* Fc[NT];
    bool cin[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const long long c = c0 + 16 * t + n;
        cin[t] = c < NC;
        const long long cc = cin[t] ? c : 0;
        Fc[t] = A.Fin + I.offF + (size_t)(cc / n2) * NV + (size_t)(cc % n2);
    }
    typedef double v4d __attribute__((ext_vector_type(4)));
    v4d acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    // kU contraction steps per round: their 5 kU operand loads are issued before the
    // MFMAs that consume them, so the L2 latencies overlap
    constexpr int kU = 4;
    for (int k0 = kbeg; k0 < kend; k0 += 4 * kU) {
        double a[kU], bv[kU][NT];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int kc = k0 + 4 * u + g;
            const bool in = kc < kend;
            a[u] = (in && row < n1) ? K1[(size_t)row * n1 + kc] : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) bv[u][t] = (in && cin[t]) ? Fc[t][(size_t)kc * n2] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (k0 + 4 * u < kend)   // wavefront-uniform: no all-zero steps past the slice
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bv[u][t], acc[t], 0, 0, 0);
    }
    if (wave > 0)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[wave - 1][t][r][lane] = acc[t][r];
    __syncthreads();
    if (wave != 0) return;
    // register r of lane group g holds output row g + 4 r of a tile, the lane's column
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const long long c = c0 + 16 * t + n;
        if (!cin[t]) continue;
        double* Yc = A.Y + (size_t)(c / n2) * NV + (size_t)(c % n2);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double v = acc[t][r];
            for (int w = 0; w < kWideThreads / kWave - 1; ++w) v += part[w][t][r][lane];
            const int i = 16 * I0 + g + 4 * r;
            if (i < n1) Yc[(size_t)i * n2] = v;
        }
    }
}

// grid: TI x ceil(2 NR n2 / kWideCols) product blocks, then nchunk prep blocks
__global__ __launch_bounds__(kWideThreads) void wide_force_prep(WideArgs A, long long tiles) {
    __shared__ double part[kWideThreads / kWave - 1][kWideCols / 16][4][kWave];
    __shared__ double sh[kWideThreads / kWave];
    if ((long long)blockIdx.x < tiles) wide_force(A, blockIdx.x, part);
    else wide_prep(A, (int)(blockIdx.x - tiles), sh);
}

// LDS rows of F an update block stages: its 256 velocities plus the rest of the first
// and last p^R rows they touch (at most 2 (Q2 - 1) more values, Q2 <= 2 kMaxQ)
constexpr int kWideRows = kWideThreads + 4 * kMaxQ;

__global__ __launch_bounds__(kWideThreads) void wide_update(WideArgs A) {
    __shared__ double sh[6 * (kWideThreads / kWave)];
    __shared__ double frow[kWideRows];
    const InstDesc& I = *A.inst;
    const double* tab = A.tab + I.offT;
    const int NR = I.NR, NV = I.NV, Q1 = I.Q1, Q2 = I.Q2, N1 = I.N1, N2 = I.N2;
    const int chunk = blockIdx.x % A.nchunk, ds = blockIdx.x / A.nchunk;   // ds = dist * NR + s
    const int dist = ds / NR, s = ds - dist * NR;
    const int k = chunk * kWideThreads + threadIdx.x;
    const bool act = k < NV;
    const int kk = act ? k : 0, vi = kk / Q2, vj = kk - vi * Q2;
    const double p1 = tab[I.tp1 + vi], p2 = tab[I.tp2 + vj];
    const double* e = A.eq + (size_t)s * kEqStride;
    const double* Fd = A.Fin + I.offF + (size_t)dist * NR * NV;
    // whole p^R rows [r0, r1] of this cell covering the block's velocities, into LDS
    const int k_lo = chunk * kWideThreads, k_hi = min(NV, k_lo + kWideThreads) - 1;
    const int r0 = k_lo / Q2, base = r0 * Q2, nrow = (k_hi / Q2 + 1) * Q2 - base;
    for (int x = threadIdx.x; x < nrow; x += kWideThreads) frow[x] = Fd[(size_t)s * NV + base + x];
    __syncthreads();
    // n_w of both walls (Eq. nw): the prep blocks' partial sums added in chunk order
    double si = 0.0, so = 0.0;
    for (int c = 0; c < A.nchunk; ++c) {
        si += A.nw[2 * c];
        so += A.nw[2 * c + 1];
    }
    const double nw_in = -si / I.den_in, nw_out = -so / I.den_out;
    const double nwi = dist ? I.T_in * nw_in : nw_in;
    const double nwo = dist ? I.T_out * nw_out : nw_out;
    const double* fin = tab + I.tfin;
    const double* fout = tab + I.tfout;
    // the reconstructed variable: f (chi form) or sqrt(g) f (f-tilde form, whose emitted
    // ghosts carry sqrt(g) of the wall)
    const bool ft = I.form == 1;
    const double* sg = tab + I.tsqg;
    auto val = [&](int c) -> double { return ft ? sg[c] * Fd[(size_t)c * NV + kk] : Fd[(size_t)c * NV + kk]; };
    // value of cell c for velocity kk: interior, emitted ghost (Eq. weno_populate) or the
    // quadratic extrapolation of the wall-bound populations (Eq. extrapol)
    auto cell = [&](int c) -> double {
        if (c >= 0 && c < NR) return val(c);
        if (c < 0) {
            if (p1 > 0.0) return ft ? I.sqg_in * (nwi * fin[kk]) : nwi * fin[kk];
            const double F1 = val(0), F2 = val(1), F3 = val(2);
            if (c == -1) return 3.0 * F1 - 3.0 * F2 + F3;
            if (c == -2) return 6.0 * F1 - 8.0 * F2 + 3.0 * F3;
            return 0.0;
        }
        if (p1 < 0.0) return ft ? I.sqg_out * (nwo * fout[kk]) : nwo * fout[kk];
        const double G1 = val(NR - 1), G2 = val(NR - 2), G3 = val(NR - 3);
        if (c == NR) return 3.0 * G1 - 3.0 * G2 + G3;
        if (c == NR + 1) return 6.0 * G1 - 8.0 * G2 + 3.0 * G3;
        return 0.0;
    };
    double m0 = 0, m1 = 0, m2 = 0, m3 = 0, rd = 0, rn = 0;
    if (act) {
        double w[7];
        for (int q = 0; q < 7; ++q) w[q] = cell(s - 3 + q);
        const bool pos = p1 > 0.0;
        const double weps = I.weno_eps;
        const double fl = weno_face<double>(pos, w[0], w[1], w[2], w[3], w[4], w[5], weps);
        const double fr = weno_face<double>(pos, w[1], w[2], w[3], w[4], w[5], w[6], weps);
        // chi form: Eq. flux_kom_R / flux_kom_eta; f-tilde form: Eq. flux_cons_R / flux_cons_eta
        // divided by sqrt(g) of the cell
        const double adv = ft ? p1 * (tab[I.tef + s + 1] * fr - tab[I.tef + s] * fl) / (I.deta * sg[s])
                              : p1 * (e[kEqGeo + 1] * fr - e[kEqGeo] * fl);
        // force: K1 F from the product launch, F Kt2^T by a short dot product along p^phi
        const double kf = A.Y[(size_t)ds * NV + kk];
        const double* Frow = frow + (vi * Q2 - base);
        const double* Kt2 = tab + I.tKt2 + (size_t)vj * Q2;
        double ktf = 0.0;
        for (int jp = 0; jp < Q2; ++jp) ktf += Kt2[jp] * Frow[jp];
        const double force = e[kEqGeo + 3] * (p2 * p2 * kf - p1 * ktf);
        // equilibrium factors g1(p_i), g2(p_j) from the cell's coefficients (side of a
        // half-range axis by the sign of the node)
        const double* c1 = e + 3 + ((I.kind1 == 1 && vi >= I.Qh1) ? N1 + 1 : 0);
        const double* c2 = e + 3 + 2 * (N1 + 1) + ((I.kind2 == 1 && vj >= I.Qh2) ? N2 + 1 : 0);
        double g1 = 0.0, g2 = 0.0;
        for (int l = 0; l <= N1; ++l) g1 += tab[I.tB1 + vi * (N1 + 1) + l] * c1[l];
        for (int l = 0; l <= N2; ++l) g2 += tab[I.tB2 + vj * (N2 + 1) + l] * c2[l];
        double fe = e[0] * g1 * g2;
        if (dist) fe *= e[1];
        const double Fc = Fd[(size_t)s * NV + kk];
        double L = -adv - force - (Fc - fe) * e[2];
        if (A.C) L += A.C[I.offF + (size_t)ds * NV + kk];
        double out;
        if (A.l_only) {
            out = L;
        } else {
            const double fn = A.Fn[I.offF + (size_t)ds * NV + kk];
            out = A.ca * fn + A.cb * Fc + A.cc * I.dt * L;
            if (A.rpart) {
                const double d = out - fn, rw = tab[I.tresW + kk];
                rd = d * d * rw;
                rn = fn * fn * rw;
            }
        }
        A.Fout[I.offF + (size_t)ds * NV + kk] = out;
        const double wo = tab[I.tWm + kk] * out;
        m0 = wo;
        if (dist == 0) {
            m1 = p1 * wo;
            m2 = p2 * wo;
            m3 = (p1 * p1 + p2 * p2) * wo;
        }
    }
    double v[6] = {m0, m1, m2, m3, rd, rn};
    block_sums<6>(v, sh);
    if (threadIdx.x == 0) {
        double* pp = A.part + (size_t)blockIdx.x * kWidePart;
        for (int q = 0; q < 6; ++q) pp[q] = v[q];
    }
}

// grid: one block per (distribution, cell); lane q < 6 adds quantity q over the chunks
__global__ __launch_bounds__(kWave) void wide_finish(WideArgs A) {
    const InstDesc& I = *A.inst;
    const double* tab = A.tab + I.offT;
    const int NR = I.NR, ds = blockIdx.x, dist = ds / NR, s = ds - dist * NR, q = threadIdx.x;
    if (q >= 6) return;
    double m = 0.0;
    for (int c = 0; c < A.nchunk; ++c) m += A.part[((size_t)ds * A.nchunk + c) * kWidePart + q];
    double* mo = A.msum_out + (size_t)(I.offC + s) * 5;
    if (q < 4) {
        if (dist == 0) mo[q] = m;
        else if (q == 0) mo[4] = m;
    } else if (A.rpart) {
        A.rpart[((size_t)(I.offC + s) * 2 + dist) * 2 + (q - 4)] = tab[I.tdchi + s] * m;
    }
}

int wide_chunks(int NV) { return (NV + kWideThreads - 1) / kWideThreads; }
size_t wide_part_doubles(int NR, int NV) { return (size_t)2 * NR * wide_chunks(NV) * kWidePart; }

hipError_t launch_wide_stage(int NR, int Q1, int Q2, hipStream_t st, const WideArgs& A) {
    const int NV = Q1 * Q2;
    if (A.nchunk != wide_chunks(NV)) return hipErrorInvalidValue;
    const long long tiles = (long long)((Q1 + 15) / 16) * (((long long)2 * NR * Q2 + kWideCols - 1) / kWideCols);
    hipLaunchKernelGGL(wide_force_prep, dim3((unsigned)(tiles + A.nchunk)), dim3(kWideThreads), 0, st, A, tiles);
    hipLaunchKernelGGL(wide_update, dim3((unsigned)(2 * NR * A.nchunk)), dim3(kWideThreads), 0, st, A);
    hipLaunchKernelGGL(wide_finish, dim3((unsigned)(2 * NR)), dim3(kWave), 0, st, A);
    return hipGetLastError();
}

}  // namespace vlb
