// Internal declarations of the expanding-channel path (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace vlb {

// Per-instance descriptor in device memory.  State block of an instance:
// F[2][NX][NL][NV] (distribution, xi cell, lambda cell, velocity k = i Q2 + j).
// Table offsets are relative to offT, in doubles.
struct ChanDesc {
    int NL, NX, Q1, Q2, NV, kind1, kind2, N1, N2, Qh1, Qh2, tau_model;
    double Kn, dt, den_lo, den_hi, weno_eps, pad0;
    long long offF, offC, offT;
    int tp1, tp2, tK1, tKt1, tK2, tKt2, tB1, tB2, tC1, tC2, tisf1, tisf2;
    int tfw, tfin, tfout, tiW;    // wall / inlet / outlet Maxwellians [2][NV] (f', f''), residual weights [NV]
                                  // (1/W_k for FP64 populations, W_k for FP32 ones scaled by 1/W_k)
    int tal, tar, tglxx, tglxl;   // per cell [NX][NL]: V^lambda factors of the left / right lambda
                                  // faces, connection coefficients G_lxx, G_lxl
    int txc, txa;                 // per (xi face, lambda row) [NX+1][NL]: V^xi = c (p^xi - a p^lambda)
    int tdlam, tdchi, tvol;       // [NL], [NX], cell volumes dchi dlambda [NX][NL]
    int strip;                    // stage-kernel traversal: lambda strips of `strip` cells, swept along xi
    int tWm;                      // [NV] W_k = w_i w_j (FP32 scaling and moment weights)
    int half;                     // 1: lambda in [0, 1], specular centreline at lambda = 0
    int ends;                     // 0: reservoir ends; 1: flow-rate ends
    int tQrow, tden, tfrow;       // flow-rate ends: prescribed row flow [2][NL] (inlet, outlet),
                                  // sum over entering k of p^y f_eq(1, u_s) [2][NL], the unit-density
                                  // Maxwellians of the rows [2][NL][2][NV] (end, row, f' / f'')
    int cartesian;                // 1: Cartesian-split momentum space (Sec. VI.G), no force terms
    int tclb;                     // cartesian: discrete metric a_p [NX], phi at the xi faces [NX + 1]
    int tgeo;                     // flow diagnostics: phi, phi' and xi at the cell centres [3][NX],
                                  // lambda faces [NL + 1] and centres [NL]
    double ipf_in, ipf_out;       // 1 / (1 + phi) at the inlet and outlet faces
};

constexpr int kChanWaves = 4;   // stage kernel: cells (one wavefront each) per block
constexpr int kChanStrip = 32;  // stage kernel: lambda-strip width of the traversal (cells)

// One stage launch covers the instances of one velocity-tile class (T1 x T2 tiles of
// 16 x 16 velocities): ilist[g] is the g-th instance of the class, whose cells occupy
// blocks [base[g], base[g+1]) in groups of kChanWaves.
struct ChanArgs {
    const ChanDesc* inst;
    const int* ilist;        // [B] instance indices of the class
    const long long* base;   // [B+1] first block of each listed instance
    int B;
    const double* tab;
    const void* Fin;         // double* (FP64 descriptors) or float* (FP32 descriptors)
    const void* Fn;
    void* Fout;
    double* rpart;           // [cells][2][2] residual partials (nullable)
    double ca, cb, cc;       // out = ca Fn + cb Fin + cc dt L[Fin]
    int l_only;              // 1: out = L[Fin]
};

// bnd = 0: the interior cells; bnd = 1: the edge bands (base[] of the matching block list)
hipError_t launch_channel_stage(int fp32, int T1, int T2, int bnd, long long nblocks, hipStream_t st,
                                const ChanArgs& A);
hipError_t launch_channel_rest(long long nelems, hipStream_t st, const ChanDesc* insts, const long long* sbase, int B,
                               const double* tab, double* F64);
// local equilibrium of the instance *inst from prof = [4][NX][NL] (n, u^lambda, u^xi, T)
hipError_t launch_channel_init_profile(long long ncells, hipStream_t st, const ChanDesc* inst, const double* tab,
                                       const double* prof, double* F64);
hipError_t launch_channel_convert(int to32, long long nelems, hipStream_t st, const ChanDesc* insts,
                                  const long long* sbase, int B, const double* tab, double* F64, float* F32);
hipError_t launch_channel_reduce(int ninst, hipStream_t st, const ChanDesc* insts, const double* tab,
                                 const double* rpart, double* resid);
hipError_t launch_channel_diag(long long ncells_total, int threads, hipStream_t st, const ChanDesc* insts,
                               const long long* cbase, int B, const double* tab, const double* F, double* diag);
// Population-kernel stage (FP64): one block of 256 threads per cell of the listed
// instances (A.ilist / A.base count cells), all vielbein (cartesian = 0) or all
// Cartesian-split (cartesian = 1)
hipError_t launch_pop_stage(int cartesian, long long ncells, hipStream_t st, const ChanArgs& A);
// flow diagnostics of the instance *inst (NX columns) from diag: out = ux, uy, P, omega
// [NX][NL] each, psi [NX][NL + 1], Pw [2][NX]
hipError_t launch_channel_fields(int NX, hipStream_t st, const ChanDesc* inst, const double* tab, const double* diag,
                                 double* out);

}  // namespace vlb
