// HIP kernels of the circular-Couette vielbein LB hot path (gfx950), FP64 and FP32.
//
// One launch = one stage of the third-order TVD Runge-Kutta scheme (Sec. III.A,
// Eq. rk3) for every instance of a batch.  A 1024-thread block holds runs of
// consecutive cells of one distribution (f' or f'') of one instance, one thread per
// velocity; each run sweeps its cells in order with a six-cell register window per
// velocity, so every population of the stage input is read from HBM once (plus a
// three-cell halo at each run end) and every output population is written once.  Per
// cell it
//   * takes n, u, T of the stage input from the moment sums its producer left
//     (Sec. IV.A, Eq. macro_red) and builds the polynomial equilibrium
//     f'_eq = n g1 g2, f''_eq = T f'_eq (Sec. IV.D, Eqs. feq_red, eq_gak_H, eq_gak_hh);
//   * computes the epsilon-free WENO-5 face flux (Sec. III.C, Eqs. weno5_flux,
//     weno5_omega, weno_sigma, Table weno), upwinded by the sign of p^R, and the chi-form
//     flux difference (Sec. V.C.1, Eqs. flux_kom_R / flux_kom_eta);
//   * applies the projected momentum derivatives of the inertial force
//     (Sec. V.A, Eq. boltz_couette_kom; kernels of Sec. IV.C) from LDS copies of the
//     cell's populations;
//   * relaxes with BGK (Eq. BGK), combines the RK stage, stores, and reduces the
//     moment sums of its output for the next stage (DPP row sums, fixed order).
// Diffuse walls (Sec. III.F, Eqs. weno_flux_eq, weno_populate, extrapol, nw): the
// runs that reach a wall recompute n_w from the wall-bound WENO flux (a half-range sum
// reduced across the run) and fill the ghost cells.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "vlb_device.h"
#include "vlb_internal.h"

namespace vlb {



// sum_i a[i] b[i], i < n (n a multiple of 4, both pointers 16-byte aligned LDS), in
// index order with 16-byte vector reads
template <typename T>
__device__ __forceinline__ T dot_lds(const T* a, const T* b, int n);
template <>
__device__ __forceinline__ float dot_lds<float>(const float* a, const float* b, int n) {
    float acc = 0.f;
    for (int i = 0; i < n; i += 4) {
        const float4 x = *reinterpret_cast<const float4*>(a + i), y = *reinterpret_cast<const float4*>(b + i);
        acc += x.x * y.x;
        acc += x.y * y.y;
        acc += x.z * y.z;
        acc += x.w * y.w;
    }
    return acc;
}
template <>
__device__ __forceinline__ double dot_lds<double>(const double* a, const double* b, int n) {
    double acc = 0.0;
    for (int i = 0; i < n; i += 2) {
        const double2 x = *reinterpret_cast<const double2*>(a + i), y = *reinterpret_cast<const double2*>(b + i);
        acc += x.x * y.x;
        acc += x.y * y.y;
    }
    return acc;
}

// The two contractions of the force term, sum_i a1[i] b1[i] (i < n1) and sum_i a2[i] b2[i]
// (i < n2), each in index order exactly as dot_lds; over the common length the reads of
// both are issued together, so that one LDS round trip serves both (FP32 kernel; the FP64
// kernel has no registers to spare and calls dot_lds twice).
__device__ __forceinline__ void dot2_lds(const float* a1, const float* b1, int n1, const float* a2,
                                         const float* b2, int n2, float& r1, float& r2) {
    float acc1 = 0.f, acc2 = 0.f;
    const int nc = n1 < n2 ? n1 : n2;
    int i = 0;
#pragma unroll 1
    for (; i < nc; i += 4) {
        const float4 x1 = *reinterpret_cast<const float4*>(a1 + i), y1 = *reinterpret_cast<const float4*>(b1 + i);
        const float4 x2 = *reinterpret_cast<const float4*>(a2 + i), y2 = *reinterpret_cast<const float4*>(b2 + i);
        acc1 += x1.x * y1.x;
        acc1 += x1.y * y1.y;
        acc1 += x1.z * y1.z;
        acc1 += x1.w * y1.w;
        acc2 += x2.x * y2.x;
        acc2 += x2.y * y2.y;
        acc2 += x2.z * y2.z;
        acc2 += x2.w * y2.w;
    }
#pragma unroll 1
    for (int j = i; j < n1; j += 4) {
        const float4 x = *reinterpret_cast<const float4*>(a1 + j), y = *reinterpret_cast<const float4*>(b1 + j);
        acc1 += x.x * y.x;
        acc1 += x.y * y.y;
        acc1 += x.z * y.z;
        acc1 += x.w * y.w;
    }
#pragma unroll 1
    for (int j = i; j < n2; j += 4) {
        const float4 x = *reinterpret_cast<const float4*>(a2 + j), y = *reinterpret_cast<const float4*>(b2 + j);
        acc2 += x.x * y.x;
        acc2 += x.y * y.y;
        acc2 += x.z * y.z;
        acc2 += x.w * y.w;
    }
    r1 = acc1;
    r2 = acc2;
}

// LDS layout of a stage block (bytes): kernel tables | two cell-row buffers (row-major
// and transposed copies per run) | two equilibrium-factor buffers | per (run, cell):
// n, T, 1/tau, equilibrium coefficients and geometry | equilibrium bases | moment and
// residual partials per wavefront (two buffers) | wall-flux partials per wavefront.
template <typename T, bool LIN = false>
struct StageLds {
    size_t ks, rows, gbuf, gbd, eqc, btab, mpart, nwpart, total;
    __host__ __device__ StageLds(int kmax) {
        auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
        ks = 0;
        rows = al(ks + (size_t)kmax * sizeof(T));
        gbuf = al(rows + 2 * (size_t)kRowElems * sizeof(T));
        gbd = al(gbuf + 2 * (size_t)kMaxRuns * kWave * sizeof(T));
        eqc = LIN ? al(gbd + 2 * (size_t)kMaxRuns * kWave * sizeof(T)) : gbd;
        btab = al(eqc + (size_t)kMaxRuns * kTileCells * kEqStride * sizeof(double));
        mpart = al(btab + (size_t)kWave * (kMaxN + 1) * sizeof(double));
        nwpart = al(mpart + 2 * (size_t)(kStageThreads / kWave) * 8 * 4 * sizeof(double));
        total = al(nwpart + (size_t)(kStageThreads / kWave) * 2 * sizeof(double));
    }
};

// LIN = true (FP32 only): the linearised stage of the defect correction.  The state is
// a correction delta about a fixed base state; advection, force and walls act on it as
// on a state (they are linear, apart from the WENO weights, which delta's own stencils
// set); the BGK term is linearised about the base: -(delta - d f_eq)/tau_base with
// d f'_eq = dn g1 g2 + n (dg1 g2 + g1 dg2), d f''_eq = T d f'_eq + dT n g1 g2, where dn, du,
// dT follow from delta's moment sums and dg = du g_u + dT g_T from the per-node factors
// of lin_prep (the variation of tau itself is left to the outer FP64 iteration).
template <typename T, bool LIN>
__device__ __forceinline__ void stage_block(const StageArgs& A, const int blk) {
    extern __shared__ double smem_d[];
    char* smem = reinterpret_cast<char*>(smem_d);
    const StageLds<T, LIN> lay(A.kmax);
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const BlockWork* bw = A.blocks + blk;
    const int inst = __builtin_amdgcn_readfirstlane(bw->inst);
    const int dist = __builtin_amdgcn_readfirstlane(bw->dist);
    const int s0 = __builtin_amdgcn_readfirstlane(bw->s0);
    const int R = __builtin_amdgcn_readfirstlane(bw->R);
    const int TC = __builtin_amdgcn_readfirstlane(bw->TC);
    const int nvpad = __builtin_amdgcn_readfirstlane(bw->nvpad);
    const InstDesc& I = A.inst[inst];
    const double* tab = A.tab + I.offT;
    const int NR = I.NR, Q1 = I.Q1, Q2 = I.Q2, NV = I.NV;

    T* Ks = reinterpret_cast<T*>(smem + lay.ks);
    T* rows = reinterpret_cast<T*>(smem + lay.rows);
    T* gbuf = reinterpret_cast<T*>(smem + lay.gbuf);
    T* gbdb = reinterpret_cast<T*>(smem + lay.gbd);
    double* eqc = reinterpret_cast<double*>(smem + lay.eqc);
    double* btab = reinterpret_cast<double*>(smem + lay.btab);
    double* mpart = reinterpret_cast<double*>(smem + lay.mpart);
    double* nwpart = reinterpret_cast<double*>(smem + lay.nwpart);

    // thread -> (run r, velocity k); nvpad is a multiple of 64, so r is wavefront-uniform
    const int r = __builtin_amdgcn_readfirstlane(t / nvpad), k = t - r * nvpad;
    const int rs0 = s0 + r * TC;
    const int rlen = r < R ? max(0, min(TC, NR - rs0)) : 0;
    const bool act = rlen > 0 && k < NV;
    const int kk = k < NV ? k : 0;
    const int vi = kk / Q2, vj = kk - vi * Q2;
    const T p1 = T(tab[I.tp1 + vi]), p2 = T(tab[I.tp2 + vj]);

    // ---- prologue: kernels into LDS (rows of stride P1 / P2, zero beyond Q1 / Q2), both
    // row buffers cleared (their padding stays zero); equilibrium coefficients of every
    // (run, cell)
    constexpr int E = sizeof(T);
    const int L1 = lds_len(Q1, E), L2 = lds_len(Q2, E);        // dot-product lengths
    const int P1 = lds_stride(Q1, E), P2 = lds_stride(Q2, E);  // LDS row strides
    const int S = row_slot(Q1, Q2, E);
    const int n1 = Q1 * P1, n2 = Q2 * P2;
    for (int x = t; x < n1 + n2; x += kStageThreads) {
        T v = T(0);
        if (x < n1) {
            const int a = x / P1, c = x - a * P1;
            if (c < Q1) v = T(tab[I.tK1 + a * Q1 + c]);
        } else {
            const int a = (x - n1) / P2, c = (x - n1) - a * P2;
            if (c < Q2) v = T(tab[I.tKt2 + a * Q2 + c]);
        }
        Ks[x] = v;
    }
    for (int x = t; x < 2 * kRowElems; x += kStageThreads) rows[x] = T(0);
    const int N1 = I.N1, N2 = I.N2;
    for (int x = t; x < R * TC; x += kStageThreads) {
        const int rr = x / TC, cc = x - rr * TC, s = s0 + rr * TC + cc;
        if (s >= NR) continue;
        const double* ms = A.msum_in + (size_t)(I.offC + s) * 5;
        double* e = eqc + (size_t)x * kEqStride;
        if constexpr (LIN) {
            // base fields, and the first-order changes of n, u, T that delta's sums carry:
            // E = sum(|p|^2 f' + f'') = 3 n T + n |u|^2
            const double* lc = A.lin_cell + (size_t)(I.offC + s) * kLinCell;
            const double n = lc[0], T_ = lc[1], u1 = lc[3], u2 = lc[4];
            const double dn = ms[0], du1 = (ms[1] - u1 * dn) / n, du2 = (ms[2] - u2 * dn) / n;
            const double dT = (ms[3] + ms[4] - (3.0 * T_ + u1 * u1 + u2 * u2) * dn - 2.0 * n * (u1 * du1 + u2 * du2)) /
                              (3.0 * n);
            e[0] = n;
            e[1] = T_;
            e[2] = lc[2];
            e[3] = dn;
            e[4] = dT;
            e[5] = du1;
            e[6] = du2;
        } else {
            const double n = ms[0], u1 = ms[1] / n, u2 = ms[2] / n;
            const double T_ = (ms[3] + ms[4] - n * (u1 * u1 + u2 * u2)) / (3.0 * n);
            e[0] = n;
            e[1] = T_;
            e[2] = 1.0 / tau_of(I.tau_model, I.Kn, n, T_);
            axis_coef(I.kind1, N1, u1, T_, tab + I.tC1, tab + I.tisf1, e + 3, e + 3 + (N1 + 1));
            axis_coef(I.kind2, N2, u2, T_, tab + I.tC2, tab + I.tisf2, e + 3 + 2 * (N1 + 1),
                      e + 3 + 2 * (N1 + 1) + (N2 + 1));
        }
        e[kEqGeo] = tab[I.tRf + s] / tab[I.tdchi + s];
        e[kEqGeo + 1] = tab[I.tRf + s + 1] / tab[I.tdchi + s];
        e[kEqGeo + 2] = tab[I.tdchi + s];
        e[kEqGeo + 3] = tab[I.tGam + s];
    }
    // equilibrium bases of both axes: rows of Q1 x (N1+1) then Q2 x (N2+1)
    const int nbt = Q1 * (N1 + 1) + Q2 * (N2 + 1);
    for (int x = t; x < nbt; x += kStageThreads)
        btab[x] = x < Q1 * (N1 + 1) ? tab[I.tB1 + x] : tab[I.tB2 + x - Q1 * (N1 + 1)];
    // node role for the per-cell factor table, taken by the run's last wavefront (its
    // first one finishes the moment sums): lane kg of it builds g1 (kg < Q1) or g2
    // (Q1 <= kg < Q1+Q2)
    const int kg = k - (nvpad - kWave);
    const double* brow = nullptr;
    int coff = -1, nb = 0;
    if (rlen > 0 && kg >= 0 && kg < Q1) {
        nb = N1 + 1;
        brow = btab + kg * nb;
        coff = 3 + ((I.kind1 == 1 && kg >= I.Qh1) ? nb : 0);
    } else if (rlen > 0 && kg >= 0 && kg < Q1 + Q2) {
        const int j = kg - Q1;
        nb = N2 + 1;
        brow = btab + Q1 * (N1 + 1) + j * nb;
        coff = 3 + 2 * (N1 + 1) + ((I.kind2 == 1 && j >= I.Qh2) ? nb : 0);
    }

    // ---- diffuse walls: n_w of Eq. nw, FP64 half-range sums reduced over the run
    const T* Fd = static_cast<const T*>(A.Fin) + I.offF + (size_t)dist * NR * NV;
    const T* Fp = static_cast<const T*>(A.Fin) + I.offF;
    const T* Fnd = static_cast<const T*>(A.Fn) + I.offF + (size_t)dist * NR * NV;
    T* Fo = static_cast<T*>(A.Fout) + I.offF + (size_t)dist * NR * NV;
    const T* Cd = A.C ? static_cast<const T*>(A.C) + I.offF + (size_t)dist * NR * NV : nullptr;
    // the cell loop's streams as range-checked buffers over this distribution's block
    const unsigned dbytes = (unsigned)((size_t)NR * NV * sizeof(T));
    const __amdgpu_buffer_rsrc_t rF = buf_rsrc(Fd, dbytes), rFn = buf_rsrc(Fnd, dbytes), rO = buf_rsrc(Fo, dbytes),
                                 rC = buf_rsrc(Cd, Cd ? dbytes : 0u);
    // element (c, k) = the lane's velocity offset kE plus the wavefront-uniform cell offset
    const unsigned kE = (unsigned)(k * sizeof(T));
    auto cofs = [&](int c) { return (unsigned)((size_t)c * NV * sizeof(T)); };
    const double* Wm = tab + I.tWm;
    const T weps = T(I.weno_eps);
    const bool near_in = rlen > 0 && rs0 < 3, near_out = rlen > 0 && rs0 + rlen > NR - 3;
    {
        double ain = 0.0, aout = 0.0;
        if (act && near_in && p1 < T(0)) {
            const T F1 = Fp[k], F2 = Fp[NV + k], F3 = Fp[2 * NV + k];
            const T g0 = T(3) * F1 - T(3) * F2 + F3, gm1 = T(6) * F1 - T(8) * F2 + T(3) * F3;
            ain = (double)p1 * Wm[k] * (double)weno5<T, LIN>(F3, F2, F1, g0, gm1, weps);
        }
        if (act && near_out && p1 > T(0)) {
            const T G1 = Fp[(size_t)(NR - 1) * NV + k], G2 = Fp[(size_t)(NR - 2) * NV + k],
                    G3 = Fp[(size_t)(NR - 3) * NV + k];
            const T g0 = T(3) * G1 - T(3) * G2 + G3, gp1 = T(6) * G1 - T(8) * G2 + T(3) * G3;
            aout = (double)p1 * Wm[k] * (double)weno5<T, LIN>(G3, G2, G1, g0, gp1, weps);
        }
        ain = wave_sum(ain);
        aout = wave_sum(aout);
        if (lane == 0) { nwpart[wave * 2] = ain; nwpart[wave * 2 + 1] = aout; }
    }
    __syncthreads();
    const int w0 = r * (nvpad / kWave), nw_waves = nvpad / kWave;
    double nw_in = 0.0, nw_out = 0.0;
    if (rlen > 0) {
        double sin_ = 0.0, sout = 0.0;
        for (int w = 0; w < nw_waves; ++w) { sin_ += nwpart[(w0 + w) * 2]; sout += nwpart[(w0 + w) * 2 + 1]; }
        if (near_in) nw_in = -sin_ / I.den_in;
        if (near_out) nw_out = -sout / I.den_out;
    }
    const T wi_scale = T(dist ? I.T_in * nw_in : nw_in);
    const T wo_scale = T(dist ? I.T_out * nw_out : nw_out);
    const double* fin = tab + I.tfin;
    const double* fout = tab + I.tfout;

    // value of cell c (0-based; ghosts outside [0, NR)) for this thread's velocity
    auto cell = [&](int c) -> T {
        if (c >= 0 && c < NR) return Fd[(size_t)c * NV + k];
        if (c < 0) {
            if (p1 > T(0)) return wi_scale * T(fin[k]);                 // Eq. weno_populate
            const T F1 = Fd[k], F2 = Fd[NV + k], F3 = Fd[2 * NV + k];
            if (c == -1) return T(3) * F1 - T(3) * F2 + F3;             // Eq. extrapol
            if (c == -2) return T(6) * F1 - T(8) * F2 + T(3) * F3;
            return T(0);
        }
        if (p1 < T(0)) return wo_scale * T(fout[k]);
        const T G1 = Fd[(size_t)(NR - 1) * NV + k], G2 = Fd[(size_t)(NR - 2) * NV + k],
                G3 = Fd[(size_t)(NR - 3) * NV + k];
        if (c == NR) return T(3) * G1 - T(3) * G2 + G3;
        if (c == NR + 1) return T(6) * G1 - T(8) * G2 + T(3) * G3;
        return T(0);
    };

    // ---- window over cells s-3 .. s+2 and the flux at the first face
    T w0v = 0, w1v = 0, w2v = 0, w3v = 0, w4v = 0, w5v = 0, fl = 0;
    const bool pos = p1 > T(0);
    if (act) {
        w0v = cell(rs0 - 3); w1v = cell(rs0 - 2); w2v = cell(rs0 - 1);
        w3v = cell(rs0);     w4v = cell(rs0 + 1); w5v = cell(rs0 + 2);
        fl = weno_face<T, LIN>(pos, w0v, w1v, w2v, w3v, w4v, w5v, weps);
    }
    // ghosts past the outer wall, which the window's leading cell reaches in the last
    // cells of the run next to it; the stage input is read-only, so they are built once
    // here and the sweep only selects them (no loads inside the sweep's ghost path, which
    // would make every cell wait for the prefetched loads)
    T gh0 = 0, gh1 = 0, gh2 = 0;
    if (act && near_out) { gh0 = cell(NR); gh1 = cell(NR + 1); gh2 = cell(NR + 2); }
    const long long offC = I.offC;

    const double dt = A.l_only ? 1.0 : I.dt;
    const T cdt = T(A.cc * dt), ca = T(A.ca), cb = T(A.cb);
    const double* resW = tab + I.tresW;
    const T* Kt = Ks + n1;
    const T* K1row = Ks + vi * P1;
    const T* Ktrow = Kt + vj * P2;
    const double pw1 = (double)p1, pw2 = (double)p2;
    // coefficients of the four moment products of the output (1, p1, p2, |p|^2), in the lane
    // order of row_sum4: this lane's quantity q = lane & 3, then q ^ 2, q ^ 1, q ^ 3
    auto mcoef = [&](int j) { return j == 0 ? 1.0 : (j == 1 ? pw1 : (j == 2 ? pw2 : pw1 * pw1 + pw2 * pw2)); };
    const int mq = lane & 3;
    const double cK1 = mcoef(mq), cK2 = mcoef(mq ^ 2), cS1 = mcoef(mq ^ 1), cS2 = mcoef(mq ^ 3);
    const double wmk = Wm[kk], rwk = resW[kk];

    // moments (and residual partials) of cell c of this run, one cell behind the sweep:
    // lane 4 q + j (q < 6, j < 4) of the run's first wavefront sums row total j of
    // quantity q over the run's wavefronts (in wavefront order); lane 4 q adds the four
    // row sums of its quad (in row order) and stores quantity q
    auto finish = [&](int c, int buf) {
        if (k >= 24 || c >= rlen) return;
        const double* mp = mpart + ((size_t)buf * (kStageThreads / kWave) + w0) * 32 + k;
        double m = 0.0;
        for (int w = 0; w < nw_waves; ++w) m += mp[(size_t)w * 32];
        const double m1 = dpp_mov<0x55>(m), m2 = dpp_mov<0xAA>(m), m3 = dpp_mov<0xFF>(m);   // quad lanes 1, 2, 3
        m = ((m + m1) + m2) + m3;
        if (k & 3) return;
        const int q = k >> 2, s = rs0 + c;
        if (q < 4) {
            if (dist == 0) A.msum_out[(size_t)(offC + s) * 5 + q] = m;
            else if (q == 0) A.msum_out[(size_t)(offC + s) * 5 + 4] = m;
        } else if (A.rpart) {
            A.rpart[((size_t)(offC + s) * 2 + dist) * 2 + (q - 4)] = eqc[(size_t)(r * TC + c) * kEqStride + kEqGeo + 2] * m;
        }
    };

    // loads issued kAhead cells before their use (the window's leading cell and F_n): the
    // cell loop is unrolled by kAhead, so slot p of the ring is read by the cells
    // c = p (mod kAhead) and refilled by them for cell c + kAhead with no register moves,
    // and a cell waits only for the loads issued kAhead cells earlier
    const bool need_fn = !A.l_only && ca != T(0);
    constexpr int kAhead = sizeof(T) == 4 ? 4 : 2;
    T pw[kAhead], fnr[kAhead], cr[LIN ? kAhead : 1];   // (the linearised stage also streams its forcing)
#pragma unroll
    for (int q = 0; q < kAhead; ++q) {
        const int x = rs0 + 3 + q;
        pw[q] = buf_load<T>(rF, (act && q < rlen && x < NR) ? kE : kBufNone, cofs(x < NR ? x : 0));
        fnr[q] = buf_load<T>(rFn, (act && need_fn && q < rlen) ? kE : kBufNone, cofs(rs0 + q));
        if constexpr (LIN) cr[q] = buf_load<T>(rC, (act && q < rlen) ? kE : kBufNone, cofs(rs0 + q));
    }

    // the run's first wavefront also finishes the previous cell's sums and its last one
    // builds the equilibrium factors; they issue ahead of the run's other wavefronts,
    // which would otherwise wait for them at every barrier
    if (rlen > 0 && ((__builtin_amdgcn_readfirstlane(k) >> 6) == 0 ||
                     (__builtin_amdgcn_readfirstlane(k) >> 6) == nw_waves - 1))
        __builtin_amdgcn_s_setprio(2);
    // each cell's output is stored at the start of the next cell, beside the prefetch
    // loads: stores count against the same wait as loads, and the loop latch waits for
    // the ring (a store issued late in the cell would be waited for there)
    T out_prev = T(0);
    unsigned st_v = kBufNone, st_s = 0;
    // linearised stage: the node factors of the run's first cell (loaded a cell ahead)
    typedef float f3v __attribute__((ext_vector_type(3)));   // (g, dg/du, dg/dT) of a node entry
    f3v lin_t4 = {0.f, 0.f, 0.f};
    // (the node-table offset made wavefront-uniform, so the resource stays in scalar registers)
    const long long offG = ((long long)__builtin_amdgcn_readfirstlane((int)(I.offG >> 32)) << 32) |
                           (unsigned)__builtin_amdgcn_readfirstlane((int)I.offG);
    const __amdgpu_buffer_rsrc_t rG =
        buf_rsrc(LIN ? A.lin_node + offG : nullptr, LIN ? (unsigned)((size_t)NR * (Q1 + Q2) * sizeof(float4)) : 0u);
    if constexpr (LIN) {
        const unsigned o = coff >= 0 ? (unsigned)(((size_t)rs0 * (Q1 + Q2) + kg) * sizeof(float4)) : kBufNone;
        lin_t4 = __builtin_bit_cast(f3v, __builtin_amdgcn_raw_buffer_load_b96(rG, o, 0, 0));
    }
#pragma unroll 1
    for (int c0 = 0; c0 < TC; c0 += kAhead) {
#pragma unroll
    for (int p = 0; p < kAhead; ++p) {
        const int c = c0 + p;
        if (c >= TC) break;
        const int buf = c & 1;
        const bool cv = act && c < rlen;
        const int s = rs0 + c;
        const T fn_cur = fnr[p];
        const T c_cur = cr[LIN ? p : 0];
        const T lead = pw[p];
        // this cell's prefetch loads refill the slots it read, each right after the slot's
        // last use, so the load can take the slot's own register
        const bool ahead = cv && c + kAhead < rlen;
        buf_store(rO, st_v, st_s, out_prev);
        st_v = kBufNone;
        T* row = rows + (size_t)buf * kRowElems + (size_t)r * 2 * S;
        T* rowT = row + S;
        T* gb = gbuf + (size_t)buf * kMaxRuns * kWave + (size_t)r * kWave;
        T* gd = gbdb + (size_t)buf * kMaxRuns * kWave + (size_t)r * kWave;
        const double* e = eqc + (size_t)(r * TC + c) * kEqStride;
        if (cv) {
            w0v = w1v; w1v = w2v; w2v = w3v; w3v = w4v; w4v = w5v;
            // s is wavefront-uniform: interior cells take a plain load
            w5v = s + 3 < NR ? lead : (s + 3 == NR ? gh0 : (s + 3 == NR + 1 ? gh1 : gh2));
            row[vi * P2 + vj] = w2v;
            rowT[vj * P1 + vi] = w2v;
        }
        pw[p] = buf_load<T>(rF, (ahead && s + 3 + kAhead < NR) ? kE : kBufNone,
                            cofs(s + 3 + kAhead < NR ? s + 3 + kAhead : 0));
        if (coff >= 0 && c < rlen) {
            if constexpr (LIN) {
                const f3v t4 = lin_t4;
                const double du = kg < Q1 ? e[5] : e[6];
                gb[kg] = T(t4.x);
                gd[kg] = T(du * (double)t4.y + e[4] * (double)t4.z);
            } else {
                double g = 0.0;
                for (int l = 0; l < nb; ++l) g += brow[l] * e[coff + l];
                gb[kg] = T(g);
            }
        }
        if constexpr (LIN) {   // the next cell's node factors (issued by every lane)
            const unsigned o = (coff >= 0 && c + 1 < rlen)
                                   ? (unsigned)(((size_t)(s + 1) * (Q1 + Q2) + kg) * sizeof(float4)) : kBufNone;
            lin_t4 = __builtin_bit_cast(f3v, __builtin_amdgcn_raw_buffer_load_b96(rG, o, 0, 0));
        }
        __syncthreads();
        if (c > 0) finish(c - 1, buf ^ 1);
        double wo = 0, rd = 0, rn = 0;
        if (cv) {
            const T fr = weno_face<T, LIN>(pos, w0v, w1v, w2v, w3v, w4v, w5v, weps);
            const T Rl = T(e[kEqGeo]), Rr = T(e[kEqGeo + 1]), gam = T(e[kEqGeo + 3]);   // R_{s-+1/2}/dchi_s
            const T adv = p1 * (Rr * fr - Rl * fl);
            T kf = T(0), ktf = T(0);
            if constexpr (sizeof(T) == 4) {
                dot2_lds(K1row, rowT + vj * P1, L1, Ktrow, row + vi * P2, L2, kf, ktf);
            } else {
                kf = dot_lds<T>(K1row, rowT + vj * P1, L1);
                ktf = dot_lds<T>(Ktrow, row + vi * P2, L2);
            }
            const T force = gam * (p2 * p2 * kf - p1 * ktf);
            T fe;
            if constexpr (LIN) {
                const T g1 = gb[vi], g2 = gb[Q1 + vj], g12 = g1 * g2;
                fe = T(e[3]) * g12 + T(e[0]) * (gd[vi] * g2 + g1 * gd[Q1 + vj]);
                if (dist) fe = T(e[1]) * fe + T(e[4] * e[0]) * g12;
            } else {
                fe = T(e[0]) * gb[vi] * gb[Q1 + vj];
                if (dist) fe = T(e[1]) * fe;
            }
            const T Fc = w2v;
            T L = -adv - force - (Fc - fe) * T(e[2]);
            if constexpr (LIN) L += c_cur;
            T out;
            if (A.l_only) {
                out = L;
            } else {
                const T fn = fn_cur;
                out = ca * fn + cb * Fc + cdt * L;
                if (A.rpart) {
                    const double d = (double)out - (double)fn;
                    rd = d * d * rwk;
                    rn = (double)fn * (double)fn * rwk;
                }
            }
            out_prev = out;
            wo = wmk * (double)out;
            fl = fr;
        }
        st_v = cv ? kE : kBufNone;   // this cell's output, stored at the top of the next cell
        st_s = cofs(s);
        fnr[p] = buf_load<T>(rFn, (ahead && need_fn) ? kE : kBufNone, cofs(s + kAhead));
        if constexpr (LIN) cr[p] = buf_load<T>(rC, ahead ? kE : kBufNone, cofs(s + kAhead));
        // row totals of the moment products (f': n, p1, p2, |p|^2 weighted; f'': n only) and
        // of the residual partials; lanes 4 q + r' hold quantity q's total of row r (the
        // finishing lanes add the rows), stored at slot 4 q + row
        double* mp = mpart + ((size_t)buf * (kStageThreads / kWave) + wave) * 32 + (lane >> 4);
        if (dist == 0) {
            const double mt = row_sum4(cK1 * wo, cK2 * wo, cS1 * wo, cS2 * wo);
            if ((lane & 15) < 4) mp[4 * mq] = mt;
        } else {
            const double m0 = row_sum(wo);
            if ((lane & 15) == 0) mp[0] = m0;
        }
        if (A.rpart) {
            rd = row_sum(rd);
            rn = row_sum(rn);
            if ((lane & 15) == 0) { mp[16] = rd; mp[20] = rn; }
        }
    }
    }
    buf_store(rO, st_v, st_s, out_prev);
    __syncthreads();
    finish(TC - 1, (TC - 1) & 1);
}

template <typename T, bool LIN>
__global__ __launch_bounds__(kStageThreads) void couette_stage(StageArgs A) {
    stage_block<T, LIN>(A, blockIdx.x);
}

// nsteps whole RK3 steps in one cooperative launch, for block lists small enough to be
// resident at once (where a step of three launches is bound by launch latency): every
// block runs its stage, then the grid synchronises (with the device-scope fence that
// makes the stage's output and moment sums visible to every XCD) before the next stage
// reads them.  Each stage is the same per-block code as couette_stage, so the result is
// bitwise that of 3 nsteps separate launches.  Every block takes the same 3 nsteps - 1
// grid barriers, and the launch is cooperative: the runtime refuses a grid whose blocks
// cannot all be resident.
template <typename T, bool LIN>
__global__ __launch_bounds__(kStageThreads) void couette_multi(MultiArgs M) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int n = 3 * M.nsteps;
    for (int q = 0; q < n; ++q) {
        const int stg = q % 3;
        StageArgs A = M.base;
        A.Fin = stg == 0 ? M.Fin[0] : (stg == 1 ? M.Fin[1] : M.Fin[2]);
        A.Fout = stg == 0 ? M.Fout[0] : (stg == 1 ? M.Fout[1] : M.Fout[2]);
        A.msum_in = stg == 0 ? M.msum_in[0] : (stg == 1 ? M.msum_in[1] : M.msum_in[2]);
        A.msum_out = stg == 0 ? M.msum_out[0] : (stg == 1 ? M.msum_out[1] : M.msum_out[2]);
        A.ca = stg == 0 ? M.ca[0] : (stg == 1 ? M.ca[1] : M.ca[2]);
        A.cb = stg == 0 ? M.cb[0] : (stg == 1 ? M.cb[1] : M.cb[2]);
        A.cc = stg == 0 ? M.cc[0] : (stg == 1 ? M.cc[1] : M.cc[2]);
        A.rpart = q == n - 1 ? M.rpart_last : nullptr;
        stage_block<T, LIN>(A, blockIdx.x);
        if (q + 1 < n) grid.sync();
    }
}

// Moment sums [n, sum p1 f', sum p2 f', sum |p|^2 f', sum f''] of a state, per cell
// (FP64 accumulation; populations weighted by Wm, 1 for unscaled FP64 states); with a
// mask, only the instances whose mask entry equals want.
template <typename T>
__global__ __launch_bounds__(256) void couette_moments(const InstDesc* insts, const WorkItem* work,
                                                       const double* tab_all, const T* F, double* msum,
                                                       const int* mask, int want) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const WorkItem* wp = work + (size_t)blockIdx.x * kWavesPerBlock + wave;
    const int inst = __builtin_amdgcn_readfirstlane(wp->inst);
    const int dist = __builtin_amdgcn_readfirstlane(wp->dist);
    const int s0 = __builtin_amdgcn_readfirstlane(wp->s0);
    const int ncell = __builtin_amdgcn_readfirstlane(wp->ncell);
    if (ncell <= 0 || dist != 0 || (mask && mask[inst] != want)) return;
    const InstDesc& I = insts[inst];
    const double* tab = tab_all + I.offT;
    const double* Wm = tab + I.tWm;
    const int NV = I.NV, Q2 = I.Q2;
    const size_t dsz = (size_t)I.NR * NV;
    for (int c = 0; c < ncell; ++c) {
        const int s = s0 + c;
        const T* fp = F + I.offF + (size_t)s * NV;
        double m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0;
        for (int k = lane; k < NV; k += kWave) {
            const int i = k / Q2, j = k - (k / Q2) * Q2;
            const double a = tab[I.tp1 + i], b = tab[I.tp2 + j];
            const double f = Wm[k] * (double)fp[k];
            m0 += f;
            m1 += a * f;
            m2 += b * f;
            m3 += (a * a + b * b) * f;
            m4 += Wm[k] * (double)fp[dsz + k];
        }
        m0 = wave_sum(m0); m1 = wave_sum(m1); m2 = wave_sum(m2); m3 = wave_sum(m3); m4 = wave_sum(m4);
        if (lane == 0) {
            double* mo = msum + (size_t)(I.offC + s) * 5;
            mo[0] = m0; mo[1] = m1; mo[2] = m2; mo[3] = m3; mo[4] = m4;
        }
    }
}

// Conversions between the FP64 state and the scaled FP32 state F/(w_i w_j) of the
// reduced-precision path, element-wise: kConvTo32 F32 = F64 / W; kConvFrom32 F64 = W F32;
// kConvAdd F64 += theta_inst W F32 (the defect correction's relaxed update); kConvZero32
// F32 = 0.
template <int MODE>
__global__ __launch_bounds__(256) void couette_convert(const InstDesc* insts32, const WorkItem* work,
                                                       const double* tab_all, double* F64, float* F32,
                                                       const double* theta) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const WorkItem* wp = work + (size_t)blockIdx.x * kWavesPerBlock + wave;
    const int inst = __builtin_amdgcn_readfirstlane(wp->inst);
    const int dist = __builtin_amdgcn_readfirstlane(wp->dist);
    const int s0 = __builtin_amdgcn_readfirstlane(wp->s0);
    const int ncell = __builtin_amdgcn_readfirstlane(wp->ncell);
    if (ncell <= 0) return;
    const InstDesc& I = insts32[inst];
    const double* W = tab_all + I.offT + I.tWm;
    const size_t base = I.offF + (size_t)dist * I.NR * I.NV;
    const double th = MODE == kConvAdd ? theta[inst] : 1.0;
    for (int c = 0; c < ncell; ++c) {
        const size_t row = base + (size_t)(s0 + c) * I.NV;
        for (int k = lane; k < I.NV; k += kWave) {
            if (MODE == kConvTo32) F32[row + k] = (float)(F64[row + k] / W[k]);
            else if (MODE == kConvFrom32) F64[row + k] = W[k] * (double)F32[row + k];
            else if (MODE == kConvAdd) F64[row + k] += th * (W[k] * (double)F32[row + k]);
            else F32[row + k] = 0.f;
        }
    }
}

// Macroscopic fields n, u^R, u^phi, T, T^{R phi}, q^R, q^phi per cell (Eq. macro_red),
// two passes over the cell's velocities (central moments about the cell velocity).
__global__ __launch_bounds__(256) void couette_diag_f64(const InstDesc* insts, const WorkItem* work,
                                                        const double* tab_all, const double* F, double* diag) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const WorkItem* wp = work + (size_t)blockIdx.x * kWavesPerBlock + wave;
    const int inst = __builtin_amdgcn_readfirstlane(wp->inst);
    const int dist = __builtin_amdgcn_readfirstlane(wp->dist);
    const int s0 = __builtin_amdgcn_readfirstlane(wp->s0);
    const int ncell = __builtin_amdgcn_readfirstlane(wp->ncell);
    if (ncell <= 0 || dist != 0) return;
    const InstDesc& I = insts[inst];
    const double* tab = tab_all + I.offT;
    const int NV = I.NV, Q2 = I.Q2;
    const size_t dsz = (size_t)I.NR * NV;
    for (int c = 0; c < ncell; ++c) {
        const int s = s0 + c;
        const double* fp = F + I.offF + (size_t)s * NV;
        double m0 = 0, m1 = 0, m2 = 0;
        for (int k = lane; k < NV; k += kWave) {
            const int i = k / Q2, j = k - (k / Q2) * Q2;
            const double f = fp[k];
            m0 += f;
            m1 += tab[I.tp1 + i] * f;
            m2 += tab[I.tp2 + j] * f;
        }
        const double n = wave_sum(m0), u1 = wave_sum(m1) / n, u2 = wave_sum(m2) / n;
        double e = 0, t12 = 0, q1 = 0, q2 = 0;
        for (int k = lane; k < NV; k += kWave) {
            const int i = k / Q2, j = k - (k / Q2) * Q2;
            const double x1 = tab[I.tp1 + i] - u1, x2 = tab[I.tp2 + j] - u2;
            const double f = fp[k], g = fp[dsz + k];
            const double xi2 = x1 * x1 + x2 * x2;
            e += xi2 * f + g;
            t12 += x1 * x2 * f;
            const double heat = 0.5 * (xi2 * f + g);
            q1 += heat * x1;
            q2 += heat * x2;
        }
        e = wave_sum(e); t12 = wave_sum(t12); q1 = wave_sum(q1); q2 = wave_sum(q2);
        if (lane == 0) {
            double* o = diag + (size_t)(I.offC + s) * 7;
            o[0] = n; o[1] = u1; o[2] = u2; o[3] = e / (3.0 * n); o[4] = t12; o[5] = q1; o[6] = q2;
        }
    }
}

// Per-instance steady-state residual and particle number, in a fixed summation order:
// r = sqrt(sum dchi (F_new - F_old)^2 / W) / (dt sqrt(sum dchi F_old^2 / W)),
// N_tot = sum_s dchi_s n_s.  One block per instance.
__global__ __launch_bounds__(256) void couette_reduce_f64(const InstDesc* insts, const double* tab_all,
                                                          const double* rpart, const double* msum,
                                                          double* resid, double* mass, int want_resid) {
    __shared__ double sh[3][256];
    const InstDesc& I = insts[blockIdx.x];
    const double* tab = tab_all + I.offT;
    double a = 0, b = 0, m = 0;
    for (int s = threadIdx.x; s < I.NR; s += blockDim.x) {
        const size_t c = (size_t)(I.offC + s);
        if (want_resid) {
            a += rpart[c * 4 + 0] + rpart[c * 4 + 2];
            b += rpart[c * 4 + 1] + rpart[c * 4 + 3];
        }
        m += tab[I.tdchi + s] * msum[c * 5];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    sh[2][threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (want_resid) resid[blockIdx.x] = sqrt(sh[0][0] / sh[1][0]) / I.dt;
        mass[blockIdx.x] = sh[2][0];
    }
}

// Warm-start fields per cell from the surrogate outputs Y[cell][4] = ((n-1) S, u^R S,
// u^phi/u_w, (T-1) S), S = 10; one block per instance.  par[inst] = (u_w, use): with use
// = 1, n is rescaled so that sum_s dchi_s n_s equals the cold start's sum_s dchi_s (n = 1)
// -- the particle number the dynamics conserve (Eq. Ntot_def) -- and u^R = 0; with use =
// 0, the cold start n = 1, u = 0, T = T_in; use < 0 leaves the instance alone.  Writes
// prof[cell][4] = (n, u^R, u^phi, T).
__global__ __launch_bounds__(256) void couette_warm_profile(const InstDesc* insts, const double* tab_all,
                                                            const float* Y, const double* par, double* prof) {
    __shared__ double sh[2][256];
    const int inst = blockIdx.x, t = threadIdx.x;
    const InstDesc& I = insts[inst];
    const double* dchi = tab_all + I.offT + I.tdchi;
    const double uw = par[2 * inst], use = par[2 * inst + 1];
    const float* y = Y + (size_t)I.offC * 4;
    double* pr = prof + (size_t)I.offC * 4;
    if (use < 0.0) return;
    if (use == 0.0) {
        for (int s = t; s < I.NR; s += 256) {
            pr[4 * s] = 1.0; pr[4 * s + 1] = 0.0; pr[4 * s + 2] = 0.0; pr[4 * s + 3] = I.T_in;
        }
        return;
    }
    double a = 0.0, c = 0.0;
    for (int s = t; s < I.NR; s += 256) {
        a += dchi[s] * (1.0 + (double)y[4 * s] / 10.0);
        c += dchi[s];
    }
    sh[0][t] = a;
    sh[1][t] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) { sh[0][t] += sh[0][t + w]; sh[1][t] += sh[1][t + w]; }
        __syncthreads();
    }
    const double scale = sh[1][0] / sh[0][0];
    for (int s = t; s < I.NR; s += 256) {
        pr[4 * s] = (1.0 + (double)y[4 * s] / 10.0) * scale;
        pr[4 * s + 1] = 0.0;
        pr[4 * s + 2] = (double)y[4 * s + 2] * uw;
        pr[4 * s + 3] = 1.0 + (double)y[4 * s + 3] / 10.0;
    }
}

// FP64 state at local equilibrium f' = n g1 g2, f'' = T f' (Sec. IV.D, Eq. feq_red) of
// the per-cell fields prof[cell][4] = (n, u^R, u^phi, T); one wavefront per work item;
// instances with par[2 inst + 1] < 0 are left alone.
__global__ __launch_bounds__(256) void couette_init_profile(const InstDesc* insts, const WorkItem* work,
                                                            const double* tab_all, const double* prof,
                                                            const double* par, double* F) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const WorkItem* wp = work + (size_t)blockIdx.x * kWavesPerBlock + wave;
    const int inst = __builtin_amdgcn_readfirstlane(wp->inst);
    const int dist = __builtin_amdgcn_readfirstlane(wp->dist);
    const int s0 = __builtin_amdgcn_readfirstlane(wp->s0);
    const int ncell = __builtin_amdgcn_readfirstlane(wp->ncell);
    if (ncell <= 0 || par[2 * inst + 1] < 0.0) return;
    const InstDesc& I = insts[inst];
    const double* tab = tab_all + I.offT;
    const int NV = I.NV, Q2 = I.Q2, N1 = I.N1, N2 = I.N2;
    double c1[2 * (kMaxN + 1)], c2[2 * (kMaxN + 1)];
    for (int c = 0; c < ncell; ++c) {
        const int s = s0 + c;
        const double* pr = prof + (size_t)(I.offC + s) * 4;
        const double n = pr[0], T_ = pr[3];
        axis_coef(I.kind1, N1, pr[1], T_, tab + I.tC1, tab + I.tisf1, c1, c1 + (N1 + 1));
        axis_coef(I.kind2, N2, pr[2], T_, tab + I.tC2, tab + I.tisf2, c2, c2 + (N2 + 1));
        double* out = F + I.offF + ((size_t)dist * I.NR + s) * NV;
        for (int k = lane; k < NV; k += kWave) {
            const int i = k / Q2, j = k - i * Q2;
            const double* e1 = c1 + ((I.kind1 == 1 && i >= I.Qh1) ? N1 + 1 : 0);
            const double* e2 = c2 + ((I.kind2 == 1 && j >= I.Qh2) ? N2 + 1 : 0);
            double g1 = 0.0, g2 = 0.0;
            for (int l = 0; l <= N1; ++l) g1 += tab[I.tB1 + i * (N1 + 1) + l] * e1[l];
            for (int l = 0; l <= N2; ++l) g2 += tab[I.tB2 + j * (N2 + 1) + l] * e2[l];
            const double v = n * g1 * g2;
            out[k] = dist ? T_ * v : v;
        }
    }
}

// Equilibrium coefficients of one axis side (as axis_coef_side) together with their
// partial derivatives with respect to the axis velocity u and the temperature T, for
// the linearised equilibrium of the defect correction (Sec. IV.D):
// full range: a_l = E[He_l(X)]/l!, X ~ N(u, T), has d a_l/du = a_{l-1} and
//   d a_l/dT = a_{l-2}/2 (He_l' = l He_{l-1}; d/dT E[f(X)] = E[f''(X)]/2);
// half range: M_s = int_0^inf x^s N(x; m, T) dx with m = +-u has
//   dM_s/dm = (M_{s+1} - m M_s)/T and dM_s/dT = (M_{s+2} - 2 m M_{s+1} + m^2 M_s)/(2 T^2) - M_s/(2 T)
//   (derivatives of the Gaussian density under the integral), and dm/du = +-1.
static __device__ __noinline__ void axis_coef_deriv(int kind, int N, double u, double T, const double* C,
                                                    const double* isf, int sg, double* co, double* cu, double* cT) {
    if (kind == 0) {
        double a[kMaxN + 1];
        a[0] = 1.0;
        if (N >= 1) a[1] = u;
        for (int l = 2; l <= N; ++l) a[l] = (u * a[l - 1] + (T - 1.0) * a[l - 2]) / l;
        for (int l = 0; l <= N; ++l) {
            co[l] = a[l] / isf[l];
            cu[l] = l >= 1 ? a[l - 1] / isf[l] : 0.0;
            cT[l] = l >= 2 ? 0.5 * a[l - 2] / isf[l] : 0.0;
        }
        return;
    }
    const double m = sg == 0 ? u : -u, sgn = sg == 0 ? 1.0 : -1.0;
    double M[kMaxN + 3];
    const double g0 = exp(-m * m / (2.0 * T)) / sqrt(2.0 * M_PI * T);
    M[0] = 0.5 * (1.0 + erf(m / sqrt(2.0 * T)));
    M[1] = m * M[0] + T * g0;
    for (int s = 2; s <= N + 2; ++s) M[s] = m * M[s - 1] + (s - 1) * T * M[s - 2];
    for (int l = 0; l <= N; ++l) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int s = 0; s <= l; ++s) {
            const double dm = (M[s + 1] - m * M[s]) / T;
            const double dT = (M[s + 2] - 2.0 * m * M[s + 1] + m * m * M[s]) / (2.0 * T * T) - M[s] / (2.0 * T);
            a += C[l * (N + 1) + s] * M[s];
            b += C[l * (N + 1) + s] * dm;
            c += C[l * (N + 1) + s] * dT;
        }
        co[l] = a;
        cu[l] = sgn * b;
        cT[l] = c;
    }
}

// Per-cell data of the linearised stage about a fixed base state (the defect
// correction's FP64 iterate): from the base state's FP64 moment sums, the cell fields
// lin_cell[cell] = (n, T, 1/tau, u1, u2) and, per node of both axes, the equilibrium
// factor g and its derivatives dg/du, dg/dT (scaled bases of the FP32 descriptor:
// w-free, as the FP32 stage builds them).  One wavefront per work item.
__global__ __launch_bounds__(256) void couette_lin_prep(const InstDesc* insts32, const WorkItem* work,
                                                        const double* tab_all, const double* msum, double* lin_cell,
                                                        float4* lin_node) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const WorkItem* wp = work + (size_t)blockIdx.x * kWavesPerBlock + wave;
    const int inst = __builtin_amdgcn_readfirstlane(wp->inst);
    const int dist = __builtin_amdgcn_readfirstlane(wp->dist);
    const int s0 = __builtin_amdgcn_readfirstlane(wp->s0);
    const int ncell = __builtin_amdgcn_readfirstlane(wp->ncell);
    if (ncell <= 0 || dist != 0) return;
    const InstDesc& I = insts32[inst];
    const double* tab = tab_all + I.offT;
    const int Q1 = I.Q1, Q2 = I.Q2, N1 = I.N1, N2 = I.N2, nq = Q1 + Q2;
    for (int c = 0; c < ncell; ++c) {
        const int s = s0 + c;
        const double* ms = msum + (size_t)(I.offC + s) * 5;
        const double n = ms[0], u1 = ms[1] / n, u2 = ms[2] / n;
        const double T = (ms[3] + ms[4] - n * (u1 * u1 + u2 * u2)) / (3.0 * n);
        if (lane == 0) {
            double* lc = lin_cell + (size_t)(I.offC + s) * kLinCell;
            lc[0] = n; lc[1] = T; lc[2] = 1.0 / tau_of(I.tau_model, I.Kn, n, T); lc[3] = u1; lc[4] = u2;
            lc[5] = lc[6] = lc[7] = 0.0;
        }
        for (int x = lane; x < nq; x += kWave) {
            const bool ax1 = x < Q1;
            const int node = ax1 ? x : x - Q1, kind = ax1 ? I.kind1 : I.kind2, N = ax1 ? N1 : N2;
            const int Qh = ax1 ? I.Qh1 : I.Qh2;
            const int sg = (kind == 1 && node >= Qh) ? 1 : 0;
            double co[kMaxN + 1], cu[kMaxN + 1], cT[kMaxN + 1];
            axis_coef_deriv(kind, N, ax1 ? u1 : u2, T, tab + (ax1 ? I.tC1 : I.tC2), tab + (ax1 ? I.tisf1 : I.tisf2),
                            sg, co, cu, cT);
            const double* B = tab + (ax1 ? I.tB1 : I.tB2) + node * (N + 1);
            double g = 0.0, gu = 0.0, gT = 0.0;
            for (int l = 0; l <= N; ++l) { g += B[l] * co[l]; gu += B[l] * cu[l]; gT += B[l] * cT[l]; }
            lin_node[(size_t)I.offG + (size_t)s * nq + x] = make_float4((float)g, (float)gu, (float)gT, 0.f);
        }
    }
}

// ------------------------------------------------------------------ host launchers
template <typename T, bool LIN>
static hipError_t launch_stage_t(int nblocks, hipStream_t st, const StageArgs& A) {
    const StageLds<T, LIN> lay(A.kmax);
    hipLaunchKernelGGL((couette_stage<T, LIN>), dim3(nblocks), dim3(kStageThreads), lay.total, st, A);
    return hipGetLastError();
}

template <typename T, bool LIN>
static hipError_t launch_multi_t(int nblocks, hipStream_t st, const MultiArgs& M) {
    const StageLds<T, LIN> lay(M.base.kmax);
    MultiArgs arg = M;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&couette_multi<T, LIN>), dim3(nblocks),
                                      dim3(kStageThreads), args, (unsigned)lay.total, st);
}

template <typename T, bool LIN>
static int multi_capacity_t(int kmax) {
    const StageLds<T, LIN> lay(kmax);
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&couette_multi<T, LIN>),
                                                     kStageThreads, lay.total) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_multi(int fp32, int nblocks, hipStream_t st, const MultiArgs& M) {
    if (fp32) return M.base.lin_cell ? launch_multi_t<float, true>(nblocks, st, M) : launch_multi_t<float, false>(nblocks, st, M);
    return launch_multi_t<double, false>(nblocks, st, M);
}

int multi_capacity(int fp32, int lin, int kmax) {
    if (fp32) return lin ? multi_capacity_t<float, true>(kmax) : multi_capacity_t<float, false>(kmax);
    return multi_capacity_t<double, false>(kmax);
}

size_t stage_lds(int kmax, int elem) {
    return elem == 4 ? StageLds<float, true>(kmax).total : StageLds<double>(kmax).total;
}

hipError_t launch_stage(int fp32, int nblocks, hipStream_t st, const StageArgs& A) {
    if (fp32) return A.lin_cell ? launch_stage_t<float, true>(nblocks, st, A) : launch_stage_t<float, false>(nblocks, st, A);
    return launch_stage_t<double, false>(nblocks, st, A);
}

hipError_t launch_moments(int fp32, int nblocks, hipStream_t st, const InstDesc* insts, const WorkItem* work,
                          const double* tab, const void* F, double* msum, const int* mask, int want) {
    if (fp32)
        hipLaunchKernelGGL(couette_moments<float>, dim3(nblocks), dim3(kWave * kWavesPerBlock), 0, st, insts, work,
                           tab, static_cast<const float*>(F), msum, mask, want);
    else
        hipLaunchKernelGGL(couette_moments<double>, dim3(nblocks), dim3(kWave * kWavesPerBlock), 0, st, insts, work,
                           tab, static_cast<const double*>(F), msum, mask, want);
    return hipGetLastError();
}

hipError_t launch_convert(int mode, int nblocks, hipStream_t st, const InstDesc* insts32, const WorkItem* work,
                          const double* tab, double* F64, float* F32, const double* theta) {
    const dim3 g(nblocks), b(kWave * kWavesPerBlock);
    switch (mode) {
        case kConvTo32:
            hipLaunchKernelGGL(couette_convert<kConvTo32>, g, b, 0, st, insts32, work, tab, F64, F32, theta);
            break;
        case kConvFrom32:
            hipLaunchKernelGGL(couette_convert<kConvFrom32>, g, b, 0, st, insts32, work, tab, F64, F32, theta);
            break;
        case kConvAdd:
            hipLaunchKernelGGL(couette_convert<kConvAdd>, g, b, 0, st, insts32, work, tab, F64, F32, theta);
            break;
        default:
            hipLaunchKernelGGL(couette_convert<kConvZero32>, g, b, 0, st, insts32, work, tab, F64, F32, theta);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_diag(int nblocks, hipStream_t st, const InstDesc* insts, const WorkItem* work,
                       const double* tab, const double* F, double* diag) {
    hipLaunchKernelGGL(couette_diag_f64, dim3(nblocks), dim3(kWave * kWavesPerBlock), 0, st, insts, work, tab, F,
                       diag);
    return hipGetLastError();
}

hipError_t launch_reduce(int ninst, hipStream_t st, const InstDesc* insts, const double* tab, const double* rpart,
                         const double* msum, double* resid, double* mass, int want_resid) {
    hipLaunchKernelGGL(couette_reduce_f64, dim3(ninst), dim3(256), 0, st, insts, tab, rpart, msum, resid, mass,
                       want_resid);
    return hipGetLastError();
}

hipError_t launch_warm_profile(int ninst, hipStream_t st, const InstDesc* insts, const double* tab, const float* Y,
                               const double* par, double* prof) {
    hipLaunchKernelGGL(couette_warm_profile, dim3(ninst), dim3(256), 0, st, insts, tab, Y, par, prof);
    return hipGetLastError();
}

hipError_t launch_init_profile(int nblocks, hipStream_t st, const InstDesc* insts, const WorkItem* work,
                               const double* tab, const double* prof, const double* par, double* F) {
    hipLaunchKernelGGL(couette_init_profile, dim3(nblocks), dim3(kWave * kWavesPerBlock), 0, st, insts, work, tab,
                       prof, par, F);
    return hipGetLastError();
}

hipError_t launch_lin_prep(int nblocks, hipStream_t st, const InstDesc* insts32, const WorkItem* work,
                           const double* tab, const double* msum, double* lin_cell, float4* lin_node) {
    hipLaunchKernelGGL(couette_lin_prep, dim3(nblocks), dim3(kWave * kWavesPerBlock), 0, st, insts32, work, tab, msum,
                       lin_cell, lin_node);
    return hipGetLastError();
}

}  // namespace vlb
