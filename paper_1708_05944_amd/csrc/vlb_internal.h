// Internal declarations of the vielbein-LB library (not part of the C ABI).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

namespace vlb {

constexpr int kMaxQ = 200;     // quadrature order per axis (nodes <= 400)
constexpr int kMaxN = 4;       // equilibrium expansion order (Eq. norder_limit: N < Q)
constexpr int kWave = 64;      // CDNA wavefront width
constexpr int kWavesPerBlock = 4;   // blocks of the auxiliary (per-wavefront work) kernels
constexpr int kStageThreads = 1024; // stage kernel block: one thread per velocity
constexpr int kMaxNV = kStageThreads;
constexpr int kTileCells = 16; // default cells per run (auxiliary kernels and stage kernel)
constexpr int kMinTile = 1, kMaxTile = 32;   // range of the stage kernel's cells per run
constexpr int kMaxRuns = 16;   // cell runs per stage block
constexpr int kEqStride = 28;  // doubles kept per cell: n, T, 1/tau, coefficients, geometry (last 4)
constexpr int kEqGeo = kEqStride - 4;   // R_{s-1/2}/dchi_s, R_{s+1/2}/dchi_s, dchi_s, Gamma_s
// LDS copies of a cell's populations for the force contractions: row-major [i][P2] and
// transposed [j][P1], and the kernel rows K1 [i][P1], Kt2 [j][P2].  A dot product runs
// over len(Q) elements (whole 16-byte vectors: 4 floats or 2 doubles, zero-padded); the
// row stride P(Q) is an odd number of 16-byte vectors, so the distinct rows one
// wavefront reads fall on distinct bank groups.  Both copies share one run slot of 2 S
// elements, S = max(Q1 P2, Q2 P1) rounded up to 4.
constexpr int kRowElems = 3136;   // per buffer: >= 2 S for every velocity set of <= kMaxNV nodes
constexpr int pad4(int x) { return (x + 3) & ~3; }
constexpr int lds_len(int Q, int elem) { return (Q + 16 / elem - 1) / (16 / elem) * (16 / elem); }
constexpr int lds_stride(int Q, int elem) {
    return ((Q + 16 / elem - 1) / (16 / elem) | 1) * (16 / elem);
}
constexpr int row_slot(int Q1, int Q2, int elem) {
    return pad4(Q1 * lds_stride(Q2, elem) > Q2 * lds_stride(Q1, elem) ? Q1 * lds_stride(Q2, elem)
                                                                      : Q2 * lds_stride(Q1, elem));
}
// the block lists serve both element sizes (a mixed batch polishes in FP64)
constexpr int row_slot_any(int Q1, int Q2) {
    return row_slot(Q1, Q2, 4) > row_slot(Q1, Q2, 8) ? row_slot(Q1, Q2, 4) : row_slot(Q1, Q2, 8);
}
constexpr int ktab_elems(int Q1, int Q2, int elem) { return Q1 * lds_stride(Q1, elem) + Q2 * lds_stride(Q2, elem); }

// Host-side tables of one momentum axis (velocity_set.cpp).
struct AxisTables {
    int kind = 0, Q = 0, N = 0, nodes = 0;
    std::vector<double> p, w;      // nodes, weights (axis ordering of Sec. IV.B)
    std::vector<double> K, Kt;     // [nodes][nodes] d/dp and d(p .)/dp kernels
    std::vector<double> B;         // [nodes][N+1] w_k phi_l(|p_k|)
    std::vector<double> C;         // [N+1][N+1] monomial coefficients of phi_l (half range)
    std::vector<double> invsqrtfact;  // 1/sqrt(l!) (full range)
};

bool build_axis(int kind, int Q, int N, AxisTables& t);
// Largest singular value of K1 (x) diag(p2^2) - diag(p1) (x) Kt2 in the quadrature-weighted
// norm (the inertial-force operator with unit connection coefficient).
double force_operator_norm(const AxisTables& a1, const AxisTables& a2);
void axis_equilibrium_host(const AxisTables& t, double u, double T, double* g);

// Per-instance descriptor in device memory.  Offsets: F in elements of the state
// buffers (instance block = [2][NR][NV]), cells in the per-cell arrays, tables in doubles.
// The FP32 path works on scaled populations F/(w_i w_j) and has its own descriptor whose
// table offsets point at rescaled tables (kernels, equilibrium bases, wall tables).
struct InstDesc {
    int NR, Q1, Q2, NV;
    int kind1, kind2, N1, N2;
    int Qh1, Qh2, tau_model, vpt;
    double Kn, dt, T_in, T_out, den_in, den_out, weno_eps;
    double deta, sqg_in, sqg_out;   // f-tilde form: cell width in eta, sqrt(g) at the walls
    long long offF, offC, offT;
    long long offG;   // node-table offset of the linearised mode (entries of 4 floats, N_R (Q1 + Q2) per instance)
    // table offsets relative to offT
    int tp1, tp2, tK1, tKt2, tB1, tB2, tC1, tC2, tisf1, tisf2;
    int tfin, tfout, tWm, tresW, tRf, tdchi, tGam;
    int form;                        // 0: chi formulation, 1: f-tilde (four-launch stage only)
    int tsqg, tef, pad0, pad1;       // f-tilde form: sqrt(g) at the cells [NR], e_eta at the faces [NR+1]
};

// One wavefront's work: cells [s0, s0 + ncell) of one distribution of one instance.
struct WorkItem {
    int inst, dist, s0, ncell;
};

// One stage-kernel block: R runs of up to TC consecutive cells starting at s0 (run r
// covers [s0 + r TC, s0 + (r+1) TC) clipped to the grid), one distribution, one
// instance; run r is held by threads [r nvpad, (r+1) nvpad), nvpad = NV rounded up to
// whole wavefronts.
struct BlockWork {
    int inst, dist, s0, R, TC, nvpad, pad0, pad1;
};

// Arguments of one RK stage launch: out = ca*Fn + cb*Fin + cc*dt*(L[Fin] + C).
// F pointers are double* (FP64 path) or float* (FP32 path).
struct StageArgs {
    const InstDesc* inst;
    const WorkItem* work;
    const double* tab;
    const void* Fin;
    const void* Fn;
    void* Fout;
    const void* C;           // constant forcing added to L (nullable)
    const double* msum_in;   // [cells][5] moment sums of Fin
    double* msum_out;        // [cells][5] moment sums of Fout
    double* rpart;           // [cells][2][2] residual partial sums (nullable)
    double ca, cb, cc;
    int l_only;              // 1: Fout = L[Fin] (dt taken as 1)
    int kmax;                // kernel-table elements reserved in LDS
    const BlockWork* blocks; // stage-kernel block list
    // linearised mode of the FP32 kernel (defect correction), both null otherwise: the
    // state is a correction delta about a fixed base state, whose per-cell fields
    // [cells][kLinCell] (n, T, 1/tau, u1, u2) and per-node equilibrium factors
    // [offG + cell (Q1 + Q2) + node] = (g, dg/du, dg/dT, 0) lin_prep wrote
    const double* lin_cell;
    const float4* lin_node;
};
constexpr int kLinCell = 8;

// Arguments of a multi-step launch: the fields the three stages of a step share, the
// per-stage buffers and RK coefficients (stage q of a step reads Fin[q], msum_in[q] and
// writes Fout[q], msum_out[q]; Fn is the step's input), and the residual partials of the
// last step's third stage (nullable).
struct MultiArgs {
    StageArgs base;
    const void* Fin[3];
    void* Fout[3];
    const double* msum_in[3];
    double* msum_out[3];
    double ca[3], cb[3], cc[3];
    double* rpart_last;
    int nsteps;
};
// modes of the FP64 <-> scaled FP32 conversion kernel
constexpr int kConvTo32 = 0, kConvFrom32 = 1, kConvAdd = 2, kConvZero32 = 3;

// Arguments of the large-velocity-set stage (one instance per launch sequence): the
// same stage as StageArgs (FP64 only), plus the instance's scratch blocks: Y [2][NR][NV]
// (K1 F), eq [NR][kEqStride], nw [nchunk][2] (wall-flux partial sums), part
// [2][NR][nchunk][8].
struct WideArgs {
    const InstDesc* inst;    // this instance's descriptor (device)
    const double* tab;
    const double* Fin;
    const double* Fn;
    double* Fout;
    const double* C;         // constant forcing added to L (nullable)
    const double* msum_in;
    double* msum_out;
    double* rpart;           // nullable
    double* Y;
    double* eq;
    double* nw;              // [nchunk][2] partial wall fluxes (inner, outer)
    double* part;
    double ca, cb, cc;
    int l_only;
    int nchunk;              // update blocks per (distribution, cell)
};
int wide_chunks(int NV);
size_t wide_part_doubles(int NR, int NV);

}  // namespace vlb
