// Host side of libvlb.so: the C ABI of include/vlb.h.  Builds velocity sets and
// Couette grids, lays out the device workspace, enqueues the stage kernels and the
// deterministic reductions, and moves data across the host/device boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/vlb.h"
#include "mlp_internal.h"
#include "vlb_internal.h"

namespace vlb {
hipError_t launch_stage(int fp32, int nblocks, hipStream_t st, const StageArgs& A);
hipError_t launch_multi(int fp32, int nblocks, hipStream_t st, const MultiArgs& M);
int multi_capacity(int fp32, int lin, int kmax);
hipError_t launch_wide_stage(int NR, int Q1, int Q2, hipStream_t st, const WideArgs& A);
size_t stage_lds(int kmax, int elem);
hipError_t launch_moments(int fp32, int nblocks, hipStream_t st, const InstDesc* insts, const WorkItem* work,
                          const double* tab, const void* F, double* msum, const int* mask = nullptr, int want = 0);
hipError_t launch_convert(int mode, int nblocks, hipStream_t st, const InstDesc* insts32, const WorkItem* work,
                          const double* tab, double* F64, float* F32, const double* theta = nullptr);
hipError_t launch_reduce(int ninst, hipStream_t st, const InstDesc* insts, const double* tab, const double* rpart,
                         const double* msum, double* resid, double* mass, int want_resid);
hipError_t launch_diag(int nblocks, hipStream_t st, const InstDesc* insts, const WorkItem* work,
                       const double* tab, const double* F, double* diag);
hipError_t launch_warm_profile(int ninst, hipStream_t st, const InstDesc* insts, const double* tab, const float* Y,
                               const double* par, double* prof);
hipError_t launch_init_profile(int nblocks, hipStream_t st, const InstDesc* insts, const WorkItem* work,
                               const double* tab, const double* prof, const double* par, double* F);
hipError_t launch_lin_prep(int nblocks, hipStream_t st, const InstDesc* insts32, const WorkItem* work,
                           const double* tab, const double* msum, double* lin_cell, float4* lin_node);
}  // namespace vlb

using namespace vlb;

namespace {

thread_local std::string g_err;

vlb_status vfail(vlb_status s, const char* fmt, va_list ap) {
    char buf[512];
    vsnprintf(buf, sizeof buf, fmt, ap);
    g_err = buf;
    return s;
}

vlb_status fail(vlb_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(s, fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(VLB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct LaunchGroup {
    int nblocks;
    int kmax;
    double pops;   // populations (2 N_R NV summed over all instances)
};

struct TimedLaunch {
    int group;
    bool fp32;
    hipEvent_t start, stop;
    double bytes;
};

struct InstHost {
    vlb_couette_desc d;
    AxisTables a1, a2;
    std::vector<double> Rf, dchi, Gam;
    int NV;
    bool wide = false;   // velocity set beyond the one-block stage kernel: the four-launch stage
    size_t wY = 0, wEq = 0, wNw = 0, wPart = 0;   // its scratch blocks (doubles into the wide region)
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace vlb {
vlb_status set_error(vlb_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(s, fmt, ap);
    va_end(ap);
    return s;
}
}  // namespace vlb

struct vlb_batch {
    int B = 0;
    hipStream_t stream = nullptr;
    std::vector<InstHost> inst;
    std::vector<InstDesc> desc;
    std::vector<WorkItem> work;        // per-wavefront list of the auxiliary kernels
    std::vector<BlockWork> blocks;     // stage-kernel blocks
    size_t max_blocks = 0;             // device capacity of the block list
    int tile = 0;                      // cells per run of the current block list
    int tile_set = kTileCells;         // cells per run chosen by vlb_batch_set_tile / vlb_batch_autotune
    std::vector<LaunchGroup> groups;
    std::vector<double> tab;
    size_t state_n = 0, ncells = 0;
    // workspace layout (byte offsets)
    size_t off_F[3], off_F32[4], off_M[3], off_rpart, off_lincell, off_linnode, off_theta, off_mask, off_resid, off_mass, off_tab, off_desc, off_desc32, off_work,
        off_diag, off_blocks, off_prof, off_wpar, off_sfeat, off_sy, off_wide, total_bytes;
    size_t wide_n = 0;                  // doubles of the large-velocity-set scratch region
    std::vector<char> active;          // instances the stage kernels advance (run_to_steady retires converged ones)
    int precision = VLB_FP64;
    bool cur32 = false;                 // the current state lives in the FP32 buffers
    long fp32_steps = 0;                // FP32 (defect-correction) steps of run_to_steady since the state was set
    bool lin = false;                   // stage launches run the linearised FP32 kernel (defect correction)
    size_t lin_nodes = 0;               // entries of the per-node table of the linearised kernel
    // learned warm start: instances still on their warm start, the step of a cold restart
    // (-1: none) and the stall window that triggers one
    std::vector<char> warm;
    std::vector<long> fallback_at;
    long stall_window = 10000;
    // run_to_steady steps since the state was replaced, and per warm instance the lowest
    // residual so far and the step count at which it was reached (kept across calls)
    long run_steps = 0;
    std::vector<double> best_res;
    std::vector<long> best_at;
    // defect correction: per-instance relaxation of the update (halved, down to 1/8, after
    // three checks in a row without a new residual low, doubled back towards 1 after eight
    // in a row with one), the lowest residual, when it was set and the run of checks
    // without / with a new low; dc64: the instance takes FP64 steps inside the correction
    // loop, launched beside the linearised FP32 ones, either on trial (kTrialChecks checks,
    // to compare the FP64 convergence rate with the correction's) or after a trial it won
    // (until it sets no new low for kDcStuck steps: then it returns to the correction)
    std::vector<double> theta, dc_best;
    std::vector<long> dc_best_at;
    std::vector<int> dc_miss, dc_hit;
    std::vector<int> dc64;
    std::vector<long> dc64_at;     // run step of the switch to FP64 steps after a won trial (-1: none)
    std::vector<long> fp32_inst;   // FP32 correction steps per instance in the current run
    std::vector<long> trial_at;    // run step at which the current FP64 trial began (-1: none)
    std::vector<long> trial_end;   // run step at which the last trial ended (-1: none yet)
    std::vector<long> trial_gap;   // steps from the end of one trial to the earliest next one
    std::vector<double> trial_r0, dc_rate;   // residual at the trial's start; the correction's rate before it
    std::vector<std::vector<std::pair<long, double>>> dc_hist;   // recent (step, residual) checks under the correction
    std::vector<BlockWork> blocks_lin, blocks_64;   // the split of `blocks` by dc64
    int n_dc64 = 0;
    std::vector<InstDesc> desc32;       // FP32 descriptors (rescaled tables)
    char* ws = nullptr;
    bool owns = false;
    double* ext_F0 = nullptr;           // caller-owned device state in place of F_n (no-allocation entry point)
    bool have_resid = false;
    bool timing = false;
    bool use_graphs = true;
    // multi-step cooperative launches for block lists of at most persist_max blocks (0:
    // never), and the resident-block capacity of each stage-kernel flavour (FP64, FP32,
    // linearised FP32; -1 until queried)
    int persist_max = 0;
    double run_seconds = 0.0;           // wall clock of the last vlb_run_to_steady
    int multi_cap[3] = {-1, -1, -1};
    hipStream_t cap_stream = nullptr;   // private stream used only to capture step graphs
    hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};   // [FP64, FP32, linearised FP32]: kGraphSteps steps
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;

    double* F(int i) { return (i == 0 && ext_F0) ? ext_F0 : (double*)(ws + off_F[i]); }
    float* F32(int i) { return (float*)(ws + off_F32[i]); }
    double* lincell() { return (double*)(ws + off_lincell); }
    double* dtheta() { return (double*)(ws + off_theta); }
    float4* linnode() { return (float4*)(ws + off_linnode); }
    InstDesc* ddesc32() { return (InstDesc*)(ws + off_desc32); }
    double* M(int i) { return (double*)(ws + off_M[i]); }
    double* rpart() { return (double*)(ws + off_rpart); }
    double* resid() { return (double*)(ws + off_resid); }
    double* massv() { return (double*)(ws + off_mass); }
    double* dtab() { return (double*)(ws + off_tab); }
    InstDesc* ddesc() { return (InstDesc*)(ws + off_desc); }
    WorkItem* dwork() { return (WorkItem*)(ws + off_work); }
    BlockWork* dblocks() { return (BlockWork*)(ws + off_blocks); }
    BlockWork* dblocks_lin() { return dblocks() + max_blocks; }
    BlockWork* dblocks_64() { return dblocks() + max_blocks + blocks_lin.size(); }
    int* dmask() { return (int*)(ws + off_mask); }
    double* prof() { return (double*)(ws + off_prof); }
    double* wpar() { return (double*)(ws + off_wpar); }
    float* sfeat() { return (float*)(ws + off_sfeat); }
    float* sy() { return (float*)(ws + off_sy); }
    double* diag() { return (double*)(ws + off_diag); }
    double* wide() { return (double*)(ws + off_wide); }
};

namespace {

bool axis_ok(const vlb_axis& a) {
    return (a.kind == 0 || a.kind == 1) && a.Q >= 1 && a.Q <= kMaxQ && a.N >= 0 && a.N < a.Q && a.N <= kMaxN;
}

// Face radii R_{s-1/2}, s = 1..N_R+1 (Sec. V.C.1; stretching Sec. III.B, Eqs. eta_def, eta_inout).
std::vector<double> faces(const vlb_couette_desc& d) {
    std::vector<double> R(d.N_R + 1);
    if (d.A == 0.0) {
        for (int s = 0; s <= d.N_R; ++s) R[s] = d.R_in + (d.R_out - d.R_in) * s / d.N_R;
    } else {
        const double A0 = std::max(d.delta, 1.0 - d.delta);
        const double el = -std::atanh(d.A * d.delta / A0), er = std::atanh(d.A * (1.0 - d.delta) / A0);
        for (int s = 0; s <= d.N_R; ++s) {
            const double eta = el + (er - el) * s / d.N_R;
            R[s] = d.R_in + (d.R_out - d.R_in) * (d.delta + A0 / d.A * std::tanh(eta));
        }
        R[0] = d.R_in;
        R[d.N_R] = d.R_out;
    }
    return R;
}

// Largest singular value of the force operator A = K1 (x) diag(p2^2) - diag(p1) (x) Kt2
// (Sec. V.A, Eq. boltz_couette_kom, with 1/R = 1) in the inner product weighted by the
// quadrature weights, where A is close to normal and this norm equals its spectral
// radius; power iteration on S^T S, S = W^{-1/2} A W^{1/2}.
double force_norm(const AxisTables& a1, const AxisTables& a2) {
    const int n1 = a1.nodes, n2 = a2.nodes, NV = n1 * n2;
    std::vector<double> s1(n1), s2(n2);
    for (int i = 0; i < n1; ++i) s1[i] = std::sqrt(a1.w[i]);
    for (int j = 0; j < n2; ++j) s2[j] = std::sqrt(a2.w[j]);
    auto K1 = [&](int i, int ip) { return a1.K[(size_t)i * n1 + ip] * s1[ip] / s1[i]; };
    auto K2 = [&](int j, int jp) { return a2.Kt[(size_t)j * n2 + jp] * s2[jp] / s2[j]; };
    std::vector<double> x(NV), y(NV), z(NV);
    for (int k = 0; k < NV; ++k) x[k] = 1.0 + 0.37 * std::sin(1.3 * k + 0.2);
    double sig = 0;
    for (int it = 0; it < 200; ++it) {
        double nx = 0;
        for (double v : x) nx += v * v;
        nx = std::sqrt(nx);
        for (double& v : x) v /= nx;
        for (int i = 0; i < n1; ++i)          // y = S x
            for (int j = 0; j < n2; ++j) {
                double a = 0, b = 0;
                for (int ip = 0; ip < n1; ++ip) a += K1(i, ip) * x[ip * n2 + j];
                for (int jp = 0; jp < n2; ++jp) b += K2(j, jp) * x[i * n2 + jp];
                y[i * n2 + j] = a2.p[j] * a2.p[j] * a - a1.p[i] * b;
            }
        for (int i = 0; i < n1; ++i)          // z = S^T y
            for (int j = 0; j < n2; ++j) {
                double a = 0, b = 0;
                for (int ip = 0; ip < n1; ++ip) a += K1(ip, i) * y[ip * n2 + j] * a2.p[j] * a2.p[j];
                for (int jp = 0; jp < n2; ++jp) b += K2(jp, j) * y[i * n2 + jp] * a1.p[i];
                z[i * n2 + j] = a - b;
            }
        double nz = 0;
        for (double v : z) nz += v * v;
        sig = std::sqrt(std::sqrt(nz));
        x.swap(z);
    }
    return sig;
}

double tau_rest(const vlb_couette_desc& d) {
    if (d.tau_model == VLB_TAU_AOKI) return d.Kn * std::sqrt(M_PI / 8.0);
    return d.Kn;
}

// Emitted-wall table f'_eq(1, (0, u), T) per velocity and the denominator of Eq. nw.
void wall_table(const InstHost& h, double u, double T, int side, std::vector<double>& tbl, double& den) {
    std::vector<double> g1(h.a1.nodes), g2(h.a2.nodes);
    axis_equilibrium_host(h.a1, 0.0, T, g1.data());
    axis_equilibrium_host(h.a2, u, T, g2.data());
    tbl.assign(h.NV, 0.0);
    den = 0.0;
    for (int i = 0; i < h.a1.nodes; ++i)
        for (int j = 0; j < h.a2.nodes; ++j) {
            const double p = h.a1.p[i];
            const bool emitted = side == 0 ? p > 0.0 : p < 0.0;
            if (!emitted) continue;
            const double v = g1[i] * g2[j];
            tbl[i * h.a2.nodes + j] = v;
            den += p * v;
        }
}

vlb_status upload_tables(vlb_batch* b) {
    HIP_TRY(hipMemcpyAsync(b->dtab(), b->tab.data(), b->tab.size() * sizeof(double), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->ddesc(), b->desc.data(), b->desc.size() * sizeof(InstDesc), hipMemcpyHostToDevice,
                           b->stream));
    if (b->precision == VLB_MIXED)
        HIP_TRY(hipMemcpyAsync(b->ddesc32(), b->desc32.data(), b->desc32.size() * sizeof(InstDesc),
                               hipMemcpyHostToDevice, b->stream));
    return VLB_OK;
}

vlb_status refresh_moments(vlb_batch* b) {
    const int nblocks = (int)(b->work.size() / kWavesPerBlock);
    if (b->cur32)
        HIP_TRY(launch_moments(1, nblocks, b->stream, b->ddesc32(), b->dwork(), b->dtab(), b->F32(0), b->M(0)));
    else
        HIP_TRY(launch_moments(0, nblocks, b->stream, b->ddesc(), b->dwork(), b->dtab(), b->F(0), b->M(0)));
    return VLB_OK;
}

// Move the current state between the FP64 buffer and the scaled FP32 buffer.
vlb_status ensure_precision(vlb_batch* b, bool want32) {
    if (b->cur32 == want32) return VLB_OK;
    if (want32 && b->precision != VLB_MIXED) return fail(VLB_ESTATE, "batch has no FP32 buffers");
    const int nblocks = (int)(b->work.size() / kWavesPerBlock);
    HIP_TRY(launch_convert(want32 ? kConvTo32 : kConvFrom32, nblocks, b->stream, b->ddesc32(), b->dwork(), b->dtab(), b->F(0),
                           b->F32(0)));
    b->cur32 = want32;
    return refresh_moments(b);
}

// A replaced state starts a new run: no FP32 steps, no steps, warm flags from `warm`
// (NULL: none), no cold restarts, no stall record.
void reset_run_state(vlb_batch* b, const int* warm) {
    b->fp32_steps = 0;
    b->run_steps = 0;
    b->warm.assign(b->B, 0);
    if (warm) for (int i = 0; i < b->B; ++i) b->warm[i] = warm[i] > 0;
    b->fallback_at.assign(b->B, -1);
    b->best_res.assign(b->B, INFINITY);
    b->best_at.assign(b->B, 0);
    b->theta.assign(b->B, 1.0);
    b->dc_miss.assign(b->B, 0);
    b->dc_hit.assign(b->B, 0);
    b->dc_best.assign(b->B, INFINITY);
    b->dc_best_at.assign(b->B, 0);
    b->dc64.assign(b->B, 0);
    b->dc64_at.assign(b->B, -1);
    b->fp32_inst.assign(b->B, 0);
    b->trial_at.assign(b->B, -1);
    b->trial_end.assign(b->B, -1);
    b->trial_gap.assign(b->B, 0);
    b->trial_r0.assign(b->B, 0.0);
    b->dc_rate.assign(b->B, 0.0);
    b->dc_hist.assign(b->B, {});
    b->n_dc64 = 0;
}

vlb_status init_from_surrogate(vlb_batch* b, const std::vector<int>& use);

vlb_status set_state_device(vlb_batch* b, const double* host) {
    HIP_TRY(hipMemcpyAsync(b->F(0), host, b->state_n * sizeof(double), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->cur32 = false;
    b->lin = false;
    b->have_resid = false;
    reset_run_state(b, nullptr);
    return refresh_moments(b);
}

// Host-side local-equilibrium state for one instance (used for initial states).
void equilibrium_state(const InstHost& h, const double* n, const double* u1, const double* u2, const double* T,
                       double* out) {
    const int NR = h.d.N_R, NV = h.NV, n1 = h.a1.nodes, n2 = h.a2.nodes;
    std::vector<double> g1(n1), g2(n2);
    for (int s = 0; s < NR; ++s) {
        axis_equilibrium_host(h.a1, u1[s], T[s], g1.data());
        axis_equilibrium_host(h.a2, u2[s], T[s], g2.data());
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                const double v = n[s] * g1[i] * g2[j];
                out[(size_t)s * NV + i * n2 + j] = v;
                out[(size_t)NR * NV + (size_t)s * NV + i * n2 + j] = T[s] * v;
            }
    }
}

vlb_status layout_and_alloc(vlb_batch* b, bool alloc, bool ext_state = false) {
    size_t off = 0;
    for (int i = 0; i < 3; ++i) {
        b->off_F[i] = off;
        if (!(i == 0 && ext_state)) off = align256(off + b->state_n * sizeof(double));
    }
    for (int i = 0; i < 4; ++i) {   // three RK buffers and the defect correction's forcing
        b->off_F32[i] = off;
        if (b->precision == VLB_MIXED) off = align256(off + b->state_n * sizeof(float));
    }
    b->off_lincell = off;
    if (b->precision == VLB_MIXED) off = align256(off + b->ncells * kLinCell * sizeof(double));
    b->off_linnode = off;
    if (b->precision == VLB_MIXED) off = align256(off + b->lin_nodes * sizeof(float4));
    b->off_theta = off;
    off = align256(off + b->B * sizeof(double));
    b->off_mask = off;
    off = align256(off + b->B * sizeof(int));
    for (int i = 0; i < 3; ++i) { b->off_M[i] = off; off = align256(off + b->ncells * 5 * sizeof(double)); }
    b->off_rpart = off; off = align256(off + b->ncells * 4 * sizeof(double));
    b->off_diag = off; off = align256(off + b->ncells * 7 * sizeof(double));
    b->off_resid = off; off = align256(off + b->B * sizeof(double));
    b->off_mass = off; off = align256(off + b->B * sizeof(double));
    b->off_tab = off; off = align256(off + b->tab.size() * sizeof(double));
    b->off_desc = off; off = align256(off + b->desc.size() * sizeof(InstDesc));
    b->off_desc32 = off; off = align256(off + b->desc32.size() * sizeof(InstDesc));
    b->off_work = off; off = align256(off + b->work.size() * sizeof(WorkItem));
    b->off_blocks = off; off = align256(off + 2 * b->max_blocks * sizeof(BlockWork));
    b->off_prof = off; off = align256(off + b->ncells * 4 * sizeof(double));
    b->off_wpar = off; off = align256(off + b->B * 2 * sizeof(double));
    b->off_sfeat = off; off = align256(off + b->ncells * 4 * sizeof(float));
    b->off_sy = off; off = align256(off + b->ncells * 4 * sizeof(float));
    b->off_wide = off; off = align256(off + b->wide_n * sizeof(double));
    b->total_bytes = off;
    if (!alloc) return VLB_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, b->total_bytes);
    if (e != hipSuccess) return fail(VLB_ENOMEM, "hipMalloc(%zu) failed: %s", b->total_bytes, hipGetErrorString(e));
    b->ws = (char*)p;
    b->owns = true;
    return VLB_OK;
}

vlb_status upload_blocks(vlb_batch* b);

vlb_status finish_setup(vlb_batch* b) {
    vlb_status st = upload_tables(b);
    if (st != VLB_OK) return st;
    HIP_TRY(hipMemcpyAsync(b->dwork(), b->work.data(), b->work.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                           b->stream));
    {
        vlb_status s2 = upload_blocks(b);
        if (s2 != VLB_OK) return s2;
    }
    // rest state n = 1, u = 0, T = T_in, built on the device exactly as the cold restart
    // of a stuck warm start
    st = init_from_surrogate(b, std::vector<int>(b->B, 0));
    if (st != VLB_OK) return st;
    reset_run_state(b, nullptr);
    return VLB_OK;
}

bool check_instance(vlb_batch* b, int inst) { return b && inst >= 0 && inst < b->B; }

// Arguments of one RK stage (or one operator application) in FP32 (f32) or FP64, the
// linearised FP32 stage of the defect correction when lin.
StageArgs stage_args(vlb_batch* b, int stage, bool last, bool l_only, bool f32, bool lin) {
    auto Fb = [&](int i) -> void* { return f32 ? (void*)b->F32(i) : (void*)b->F(i); };
    StageArgs A;
    A.inst = f32 ? b->ddesc32() : b->ddesc();
    A.work = b->dwork();
    A.tab = b->dtab();
    A.rpart = nullptr;
    A.C = nullptr;
    A.lin_cell = nullptr;
    A.lin_node = nullptr;
    if (lin && f32) {   // linearised FP32 stage about the defect correction's base state
        A.lin_cell = b->lincell();
        A.lin_node = b->linnode();
        A.C = b->F32(3);
    }
    A.l_only = l_only ? 1 : 0;
    if (l_only) {
        A.Fin = Fb(0); A.Fn = Fb(0); A.Fout = Fb(1);
        A.msum_in = b->M(0); A.msum_out = b->M(1);
        A.ca = 0.0; A.cb = 0.0; A.cc = 1.0;
    } else if (stage == 0) {
        A.Fin = Fb(0); A.Fn = Fb(0); A.Fout = Fb(1);
        A.msum_in = b->M(0); A.msum_out = b->M(1);
        A.ca = 0.0; A.cb = 1.0; A.cc = 1.0;
    } else if (stage == 1) {
        A.Fin = Fb(1); A.Fn = Fb(0); A.Fout = Fb(2);
        A.msum_in = b->M(1); A.msum_out = b->M(2);
        A.ca = 0.75; A.cb = 0.25; A.cc = 0.25;
    } else {
        A.Fin = Fb(2); A.Fn = Fb(0); A.Fout = Fb(0);
        A.msum_in = b->M(2); A.msum_out = b->M(0);
        A.ca = 1.0 / 3.0; A.cb = 2.0 / 3.0; A.cc = 2.0 / 3.0;
        if (last && !A.lin_cell) A.rpart = b->rpart();
    }
    return A;
}

// One RK stage (or one operator application) on the current precision's buffers.  In the
// defect correction, instances that fell back to FP64 (dc64) take their FP64 stage in a
// second launch beside the linearised FP32 one.
vlb_status run_stage(vlb_batch* b, int stage, bool last, bool l_only) {
    const bool f32 = b->cur32;
    if (b->lin && f32 && b->n_dc64 > 0 && !l_only) {
        const LaunchGroup& g = b->groups[0];
        StageArgs A = stage_args(b, stage, last, false, true, true);
        A.blocks = b->dblocks_lin();
        A.kmax = g.kmax;
        if (!b->blocks_lin.empty()) HIP_TRY(launch_stage(1, (int)b->blocks_lin.size(), b->stream, A));
        StageArgs A64 = stage_args(b, stage, last, false, false, false);
        A64.blocks = b->dblocks_64();
        A64.kmax = g.kmax;
        if (!b->blocks_64.empty()) HIP_TRY(launch_stage(0, (int)b->blocks_64.size(), b->stream, A64));
        return VLB_OK;
    }
    const StageArgs A = stage_args(b, stage, last, l_only, f32, b->lin);
    const double values = (l_only || stage == 0) ? 2.0 : 3.0;   // algorithmic HBM values per population
    const double elem = f32 ? sizeof(float) : sizeof(double);
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const LaunchGroup& g = b->groups[gi];
        StageArgs G = A;
        G.blocks = b->dblocks();
        G.kmax = g.kmax;
        TimedLaunch t{};
        if (b->timing) {
            for (hipEvent_t* e : {&t.start, &t.stop}) {
                if (b->event_pool.empty()) {
                    HIP_TRY(hipEventCreate(e));
                } else {
                    *e = b->event_pool.back();
                    b->event_pool.pop_back();
                }
            }
            HIP_TRY(hipEventRecord(t.start, b->stream));
        }
        if (g.nblocks > 0) HIP_TRY(launch_stage(f32 ? 1 : 0, g.nblocks, b->stream, G));
        if (b->timing) {
            HIP_TRY(hipEventRecord(t.stop, b->stream));
            t.group = (int)gi;
            t.fp32 = f32;
            t.bytes = values * g.pops * elem;
            b->timed.push_back(t);
        }
    }
    // instances with large velocity sets (FP64 only): four launches each
    for (int i = 0; i < b->B; ++i) {
        const InstHost& h = b->inst[i];
        if (!h.wide || (!b->active.empty() && !b->active[i])) continue;
        WideArgs W;
        W.inst = b->ddesc() + i;
        W.tab = b->dtab();
        W.Fin = static_cast<const double*>(A.Fin);
        W.Fn = static_cast<const double*>(A.Fn);
        W.Fout = static_cast<double*>(A.Fout);
        W.C = nullptr;
        W.msum_in = A.msum_in;
        W.msum_out = A.msum_out;
        W.rpart = A.rpart;
        W.Y = b->wide() + h.wY;
        W.eq = b->wide() + h.wEq;
        W.nw = b->wide() + h.wNw;
        W.part = b->wide() + h.wPart;
        W.ca = A.ca; W.cb = A.cb; W.cc = A.cc;
        W.l_only = A.l_only;
        W.nchunk = wide_chunks(h.NV);
        HIP_TRY(launch_wide_stage(h.d.N_R, h.a1.nodes, h.a2.nodes, b->stream, W));
    }
    return VLB_OK;
}

constexpr int kGraphSteps = 10;
constexpr long kDcStuck = 20000;    // steps without a new residual low that return an instance to the correction
constexpr int kTrialChecks = 5;     // checks of an FP64 trial
constexpr int kRateChecks = 10;     // checks over which the correction's rate is measured
constexpr int kTrialGap = 4;        // trial lengths between trials of an instance (doubled after each lost one)
constexpr double kTrialGain = 1.5;  // the FP64 rate must beat the correction's by this factor to be kept
constexpr double kTrialDrop = 2;    // ... and the residual fall by at least this factor over the trial
constexpr double kSlowDecade = 10;  // a correction slower than one decade per kRateChecks checks is put on trial

void drop_graphs(vlb_batch* b) {
    for (hipGraphExec_t& g : b->graph)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

// Capture kGraphSteps RK3 steps (3 stage launches each, no residual) of the current
// precision into an executable graph, on a private stream.
vlb_status capture_steps(vlb_batch* b, hipGraphExec_t* out) {
    if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    hipStream_t user = b->stream;
    b->stream = b->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    vlb_status st = VLB_OK;
    if (e == hipSuccess) {
        for (int it = 0; it < kGraphSteps && st == VLB_OK; ++it)
            for (int stage = 0; stage < 3 && st == VLB_OK; ++stage) st = run_stage(b, stage, false, false);
        e = hipStreamEndCapture(b->cap_stream, &g);
    }
    b->stream = user;
    if (st != VLB_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return fail(VLB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(VLB_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    return VLB_OK;
}

// Stage-kernel blocks for cell runs of about `tile` cells: per instance and distribution,
// the grid is cut into runs of equal length <= tile; a block holds R runs (one group of
// whole wavefronts per run, R <= kMaxRuns and R * tile <= kMaxRuns * kTileCells); the
// heaviest blocks go first so the tail of a launch is made of small blocks.
void build_blocks(vlb_batch* b, int tile) {
    b->blocks.clear();
    for (int i = 0; i < b->B; ++i) {
        if ((!b->active.empty() && !b->active[i]) || b->inst[i].wide) continue;
        const InstDesc& D = b->desc[i];
        const int nruns = (D.NR + tile - 1) / tile;
        const int per = (D.NR + nruns - 1) / nruns;
        const int nvpad = (D.NV + kWave - 1) / kWave * kWave;
        const int rmax = std::max(1, std::min({kMaxRuns, kStageThreads / nvpad, kMaxRuns * kTileCells / per,
                                               kRowElems / (2 * row_slot_any(D.Q1, D.Q2))}));
        for (int dist = 0; dist < 2; ++dist)
            for (int r0 = 0; r0 < nruns; r0 += rmax)
                b->blocks.push_back({i, dist, r0 * per, std::min(rmax, nruns - r0), per, nvpad, 0, 0});
    }
    std::stable_sort(b->blocks.begin(), b->blocks.end(), [&](const BlockWork& x, const BlockWork& y) {
        const double wx = (double)x.R * x.TC * b->desc[x.inst].NV, wy = (double)y.R * y.TC * b->desc[y.inst].NV;
        return wx > wy;
    });
    for (LaunchGroup& g : b->groups) g.nblocks = (int)b->blocks.size();
    b->tile = tile;
    b->blocks_lin.clear();
    b->blocks_64.clear();
    for (const BlockWork& w : b->blocks)
        ((b->dc64.size() == (size_t)b->B && b->dc64[w.inst]) ? b->blocks_64 : b->blocks_lin).push_back(w);
}

// Cells per run for the instances still active in run_to_steady: the chosen length while
// its block list fills the CUs (one 1024-thread block each), else the longest shorter one
// that does (down to kMinTile): a partly filled launch costs the latency of its longest
// block, which is the cell-run length.  Leaves the block list built for the result.
int active_tile(vlb_batch* b) {
    constexpr size_t kFillBlocks = 256;
    for (int t = b->tile_set; t > kMinTile; --t) {
        build_blocks(b, t);
        if (b->blocks.size() >= kFillBlocks) return t;
    }
    build_blocks(b, kMinTile);
    return kMinTile;
}

vlb_status upload_blocks(vlb_batch* b) {
    HIP_TRY(hipMemcpyAsync(b->dblocks(), b->blocks.data(), b->blocks.size() * sizeof(BlockWork),
                           hipMemcpyHostToDevice, b->stream));
    if (b->n_dc64 > 0) {   // the linearised / FP64 split of the defect correction
        HIP_TRY(hipMemcpyAsync(b->dblocks_lin(), b->blocks_lin.data(), b->blocks_lin.size() * sizeof(BlockWork),
                               hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipMemcpyAsync(b->dblocks_64(), b->blocks_64.data(), b->blocks_64.size() * sizeof(BlockWork),
                               hipMemcpyHostToDevice, b->stream));
    }
    drop_graphs(b);   // captured launches carry the old grid size
    return VLB_OK;
}

constexpr long kMultiChunk = 2000;   // steps per multi-step launch

// The multi-step launch applies: a single block list of at most persist_max blocks that
// the device can hold resident at once, no large-velocity-set instance running, no
// FP64 / linearised split of the defect correction, no per-launch timing.
bool multi_ok(vlb_batch* b) {
    if (b->persist_max <= 0 || b->timing || b->groups.size() != 1) return false;
    if (b->lin && b->n_dc64 > 0) return false;
    const int nb = (int)b->blocks.size();
    if (nb <= 0 || nb > b->persist_max) return false;
    for (int i = 0; i < b->B; ++i)
        if (b->inst[i].wide && (b->active.empty() || b->active[i])) return false;
    const int key = b->cur32 ? (b->lin ? 2 : 1) : 0;
    if (b->multi_cap[key] < 0) b->multi_cap[key] = multi_capacity(b->cur32, b->lin, b->groups[0].kmax);
    return nb <= b->multi_cap[key];
}

// nsteps RK3 steps in multi-step launches of at most kMultiChunk steps (the residual
// partials taken in the last step's third stage, as step_current's last plain step does).
vlb_status step_multi(vlb_batch* b, long nsteps) {
    MultiArgs M{};
    for (int q = 0; q < 3; ++q) {
        const StageArgs S = stage_args(b, q, false, false, b->cur32, b->lin);
        if (q == 0) M.base = S;
        M.Fin[q] = S.Fin;
        M.Fout[q] = S.Fout;
        M.msum_in[q] = S.msum_in;
        M.msum_out[q] = S.msum_out;
        M.ca[q] = S.ca;
        M.cb[q] = S.cb;
        M.cc[q] = S.cc;
    }
    M.base.blocks = b->dblocks();
    M.base.kmax = b->groups[0].kmax;
    const int nb = (int)b->blocks.size();
    for (long left = nsteps; left > 0;) {
        const long n = std::min(left, kMultiChunk);
        M.nsteps = (int)n;
        M.rpart_last = (n == left && !b->lin) ? b->rpart() : nullptr;
        HIP_TRY(launch_multi(b->cur32 ? 1 : 0, nb, b->stream, M));
        left -= n;
    }
    if (!b->lin) {
        HIP_TRY(launch_reduce(b->B, b->stream, b->cur32 ? b->ddesc32() : b->ddesc(), b->dtab(), b->rpart(), b->M(0),
                              b->resid(), b->massv(), 1));
        b->have_resid = true;
    }
    return VLB_OK;
}

vlb_status step_current(vlb_batch* b, long nsteps) {
    if (nsteps >= 2 && multi_ok(b)) return step_multi(b, nsteps);
    // all but the last step: replay captured chunks of kGraphSteps steps
    if (b->use_graphs && !b->timing && nsteps > kGraphSteps) {
        hipGraphExec_t& g = b->graph[b->cur32 ? (b->lin ? 2 : 1) : 0];
        if (!g) {
            vlb_status s = capture_steps(b, &g);
            if (s != VLB_OK) return s;
        }
        while (nsteps > kGraphSteps) {
            HIP_TRY(hipGraphLaunch(g, b->stream));
            nsteps -= kGraphSteps;
        }
    }
    for (long it = 0; it < nsteps; ++it) {
        const bool last = it + 1 == nsteps;
        for (int st = 0; st < 3; ++st) {
            vlb_status s = run_stage(b, st, last, false);
            if (s != VLB_OK) return s;
        }
        if (last && !b->lin) {
            HIP_TRY(launch_reduce(b->B, b->stream, b->cur32 ? b->ddesc32() : b->ddesc(), b->dtab(), b->rpart(), b->M(0),
                                  b->resid(), b->massv(), 1));
            b->have_resid = true;
        }
    }
    return VLB_OK;
}

vlb_status read_residual(vlb_batch* b, double* r) {
    HIP_TRY(hipMemcpyAsync(r, b->resid(), b->B * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (int i = 0; i < b->B; ++i)
        if (!std::isfinite(r[i])) return fail(VLB_ENONFINITE, "non-finite residual in instance %d", i);
    return VLB_OK;
}

// One defect-correction pass of the mixed path, on the FP64 iterate F64 in F(0) (with
// its moment sums in M(0)): the FP64 defect R = L64[F64]; then m RK3 steps in FP32 of the
// correction equation d delta/dt = R + J delta from delta = 0, where J is the FP32
// operator linearised about F64 (linearised FP32 stage kernel); then F64 += delta.  The
// correction is stored and streamed in FP32 at its own scale, so its rounding is
// relative to delta, not to F; at a fixed point of the outer iteration R = 0, i.e. the
// FP64 steady state.  Leaves F(0) and M(0) current in FP64.
vlb_status defect_correction(vlb_batch* b, long m) {
    const int nblocks = (int)(b->work.size() / kWavesPerBlock);
    HIP_TRY(launch_lin_prep(nblocks, b->stream, b->ddesc32(), b->dwork(), b->dtab(), b->M(0), b->lincell(),
                            b->linnode()));
    vlb_status s = run_stage(b, 0, false, true);   // R = L64[F64] into F(1)
    if (s != VLB_OK) return s;
    HIP_TRY(launch_convert(kConvTo32, nblocks, b->stream, b->ddesc32(), b->dwork(), b->dtab(), b->F(1), b->F32(3)));
    HIP_TRY(launch_convert(kConvZero32, nblocks, b->stream, b->ddesc32(), b->dwork(), b->dtab(), b->F(0), b->F32(0)));
    HIP_TRY(launch_moments(1, nblocks, b->stream, b->ddesc32(), b->dwork(), b->dtab(), b->F32(0), b->M(0)));
    if (b->n_dc64 > 0)   // instances stepping in FP64 keep the moment sums of their FP64 state
        HIP_TRY(launch_moments(0, nblocks, b->stream, b->ddesc(), b->dwork(), b->dtab(), b->F(0), b->M(0), b->dmask(),
                               1));
    b->cur32 = true;
    b->lin = true;
    s = step_current(b, m);
    b->cur32 = false;
    b->lin = false;
    if (s != VLB_OK) return s;
    HIP_TRY(hipMemcpyAsync(b->dtheta(), b->theta.data(), b->B * sizeof(double), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(launch_convert(kConvAdd, nblocks, b->stream, b->ddesc32(), b->dwork(), b->dtab(), b->F(0), b->F32(0),
                           b->dtheta()));
    b->have_resid = false;
    return refresh_moments(b);
}

}  // namespace

extern "C" {

const char* vlb_status_string(vlb_status s) {
    switch (s) {
        case VLB_OK: return "ok";
        case VLB_EINVAL: return "invalid argument";
        case VLB_ENOMEM: return "out of memory";
        case VLB_EDEVICE: return "device error";
        case VLB_ESTATE: return "invalid state";
        case VLB_ENOTCONV: return "not converged";
        case VLB_ENONFINITE: return "non-finite value";
        case VLB_EUNSTABLE: return "unstable time step";
    }
    return "unknown status";
}

const char* vlb_last_error(void) { return g_err.c_str(); }

vlb_status vlb_axis_tables(vlb_axis ax, double* p, double* w, double* K, double* Kt) {
    if (!axis_ok(ax)) return fail(VLB_EINVAL, "invalid axis (kind=%d Q=%d N=%d)", ax.kind, ax.Q, ax.N);
    AxisTables t;
    if (!build_axis(ax.kind, ax.Q, ax.N, t)) return fail(VLB_EINVAL, "axis construction failed");
    if (p) std::memcpy(p, t.p.data(), t.p.size() * sizeof(double));
    if (w) std::memcpy(w, t.w.data(), t.w.size() * sizeof(double));
    if (K) std::memcpy(K, t.K.data(), t.K.size() * sizeof(double));
    if (Kt) std::memcpy(Kt, t.Kt.data(), t.Kt.size() * sizeof(double));
    return VLB_OK;
}

vlb_status vlb_batch_create_couette(vlb_batch** out, int B, const vlb_couette_desc* descs, int precision,
                                    void* hip_stream, int defer_alloc) {
    if (!out || B < 1 || !descs) return fail(VLB_EINVAL, "need out, B >= 1 and descriptors");
    *out = nullptr;
    if (precision != VLB_FP64 && precision != VLB_MIXED) return fail(VLB_EINVAL, "unsupported precision %d", precision);
    vlb_batch* b = new (std::nothrow) vlb_batch;
    if (!b) return fail(VLB_ENOMEM, "host allocation failed");
    b->B = B;
    b->precision = precision;
    b->stream = (hipStream_t)hip_stream;
    b->inst.resize(B);
    b->desc.resize(B);
    if (precision == VLB_MIXED) b->desc32.resize(B);
    std::map<std::tuple<int, int, int>, AxisTables> cache;
    size_t offF = 0, offC = 0;
    for (int i = 0; i < B; ++i) {
        const vlb_couette_desc& d = descs[i];
        if (!(d.N_R >= 3 && d.R_in > 0 && d.R_out > d.R_in && d.Kn > 0 && d.dt >= 0 && d.A >= 0 && d.A < 1 &&
              d.delta >= 0 && d.delta <= 1 && d.T_in > 0 && d.T_out > 0 && d.tau_model >= 0 && d.tau_model <= 2 &&
              axis_ok(d.ax1) && axis_ok(d.ax2) && (d.dt > 0 || d.cfl > 0) && d.weno_eps >= 0 &&
              std::isfinite(d.weno_eps) && (d.form == 0 || d.form == 1))) {
            delete b;
            return fail(VLB_EINVAL, "invalid descriptor for instance %d", i);
        }
        InstHost& h = b->inst[i];
        h.d = d;
        for (int ax = 0; ax < 2; ++ax) {
            const vlb_axis& a = ax == 0 ? d.ax1 : d.ax2;
            auto key = std::make_tuple(a.kind, a.Q, a.N);
            auto it = cache.find(key);
            if (it == cache.end()) {
                AxisTables t;
                if (!build_axis(a.kind, a.Q, a.N, t)) { delete b; return fail(VLB_EINVAL, "axis build failed"); }
                it = cache.emplace(key, std::move(t)).first;
            }
            (ax == 0 ? h.a1 : h.a2) = it->second;
        }
        h.NV = h.a1.nodes * h.a2.nodes;
        // the one-block stage kernel holds a cell's velocities in one block and both kernel
        // tables in LDS; larger sets take the four-launch stage (FP64)
        h.wide = d.form == 1 || h.NV > kMaxNV || h.a1.nodes + h.a2.nodes > kWave ||
                 2 * row_slot_any(h.a1.nodes, h.a2.nodes) > kRowElems ||
                 stage_lds(pad4(std::max(ktab_elems(h.a1.nodes, h.a2.nodes, 4), ktab_elems(h.a1.nodes, h.a2.nodes, 8))),
                           sizeof(double)) > 160 * 1024;
        if (h.wide && precision == VLB_MIXED) {
            delete b;
            return fail(VLB_EINVAL, "instance %d: %d velocities (%d + %d nodes) or the f-tilde form run in FP64 only",
                        i, h.NV, h.a1.nodes, h.a2.nodes);
        }
        h.Rf = faces(d);
        h.dchi.resize(d.N_R);
        h.Gam.resize(d.N_R);
        for (int s = 0; s < d.N_R; ++s) {
            h.dchi[s] = 0.5 * (h.Rf[s + 1] * h.Rf[s + 1] - h.Rf[s] * h.Rf[s]);   // chi = R^2/2
            h.Gam[s] = 2.0 / (h.Rf[s + 1] + h.Rf[s]);                              // 1/R of the force, cell value
        }
        // time-step limits: advection CFL (number 1), the force operator on the imaginary
        // axis of the RK3 stability region (|lambda dt| <= sqrt(3)), and the BGK relaxation
        double pmax = 0;
        for (double v : h.a1.p) pmax = std::max(pmax, std::fabs(v));
        double dt_adv = 1e300, gmax = 0;
        for (int s = 0; s < d.N_R; ++s) {
            dt_adv = std::min(dt_adv, h.dchi[s] / (h.Rf[s + 1] * pmax));
            gmax = std::max(gmax, h.Gam[s]);
        }
        const double rho_force = gmax * force_norm(h.a1, h.a2);
        const double dt1 = 1.0 / (1.0 / dt_adv + rho_force / std::sqrt(3.0));
        double dt = d.dt;
        if (dt == 0.0) {
            dt = std::min(d.cfl * dt1, 2.0 * tau_rest(d));
        } else if (dt > dt1 || dt > 2.5 * tau_rest(d)) {
            delete b;
            return fail(VLB_EUNSTABLE, "instance %d: dt=%g exceeds the stability limit %g (advection %g, force %g) "
                        "or 2.5 tau=%g", i, dt, dt1, dt_adv, std::sqrt(3.0) / rho_force, 2.5 * tau_rest(d));
        }

        InstDesc& D = b->desc[i];
        std::memset(&D, 0, sizeof D);
        D.NR = d.N_R;
        D.Q1 = h.a1.nodes;
        D.Q2 = h.a2.nodes;
        D.NV = h.NV;
        D.kind1 = h.a1.kind; D.kind2 = h.a2.kind;
        D.N1 = h.a1.N; D.N2 = h.a2.N;
        D.Qh1 = h.a1.Q; D.Qh2 = h.a2.Q;
        D.tau_model = d.tau_model;
        D.vpt = (h.NV + kWave - 1) / kWave;
        D.Kn = d.Kn;
        D.weno_eps = d.weno_eps;
        D.dt = dt;
        D.T_in = d.T_in;
        D.T_out = d.T_out;
        D.offF = (long long)offF;
        D.offC = (long long)offC;
        D.offG = (long long)b->lin_nodes;
        b->lin_nodes += (size_t)d.N_R * (h.a1.nodes + h.a2.nodes);
        D.offT = (long long)b->tab.size();
        auto put = [&](const std::vector<double>& v) {
            int o = (int)(b->tab.size() - D.offT);
            b->tab.insert(b->tab.end(), v.begin(), v.end());
            return o;
        };
        D.tp1 = put(h.a1.p); D.tp2 = put(h.a2.p);
        D.tK1 = put(h.a1.K); D.tKt2 = put(h.a2.Kt);
        D.tB1 = put(h.a1.B); D.tB2 = put(h.a2.B);
        D.tC1 = put(h.a1.C); D.tC2 = put(h.a2.C);
        D.tisf1 = put(h.a1.invsqrtfact); D.tisf2 = put(h.a2.invsqrtfact);
        std::vector<double> tin, tout;
        wall_table(h, d.u_in, d.T_in, 0, tin, D.den_in);
        wall_table(h, d.u_out, d.T_out, 1, tout, D.den_out);
        D.tfin = put(tin);
        D.tfout = put(tout);
        std::vector<double> W(h.NV), invW(h.NV), ones(h.NV, 1.0);
        for (int a = 0; a < h.a1.nodes; ++a)
            for (int c = 0; c < h.a2.nodes; ++c) {
                W[a * h.a2.nodes + c] = h.a1.w[a] * h.a2.w[c];
                invW[a * h.a2.nodes + c] = 1.0 / W[a * h.a2.nodes + c];
            }
        D.tWm = put(ones);       // stored populations are the weighted f_ij themselves
        D.tresW = put(invW);     // ||F||_W^2 = sum F^2 / W
        D.tRf = put(h.Rf);
        D.tdchi = put(h.dchi);
        D.tGam = put(h.Gam);
        D.form = d.form;
        if (d.form == 1) {
            // f-tilde metric: sqrt(g) = R R'(eta) at the cell centres (eta midpoints), e_eta^eta =
            // 1/R'(eta) at the faces, the cell width in eta and sqrt(g) at the walls; equal
            // cells take eta = R.  The emitted wall ghosts hold sqrt(g_wall) n_w f_eq, so the
            // zero-flux density divides by sqrt(g_wall) as well.
            std::vector<double> sqg(d.N_R), ef(d.N_R + 1);
            if (d.A == 0.0) {
                for (int s = 0; s < d.N_R; ++s) sqg[s] = 0.5 * (h.Rf[s] + h.Rf[s + 1]);
                for (int s = 0; s <= d.N_R; ++s) ef[s] = 1.0;
                D.deta = (d.R_out - d.R_in) / d.N_R;
                D.sqg_in = d.R_in;
                D.sqg_out = d.R_out;
            } else {
                const long double A0 = std::max(d.delta, 1.0 - d.delta), AA = d.A, span = d.R_out - d.R_in;
                const long double el = -std::atanh(AA * d.delta / A0), er = std::atanh(AA * (1.0L - d.delta) / A0);
                const long double de = (er - el) / d.N_R;
                auto Rof = [&](long double e) { return (long double)d.R_in + span * ((long double)d.delta + A0 / AA * std::tanh(e)); };
                auto dRof = [&](long double e) { const long double c = std::cosh(e); return span * A0 / (AA * c * c); };
                for (int s = 0; s < d.N_R; ++s) {
                    const long double e = el + (s + 0.5L) * de;
                    sqg[s] = (double)(Rof(e) * dRof(e));
                }
                for (int s = 0; s <= d.N_R; ++s) ef[s] = (double)(1.0L / dRof(el + s * de));
                D.deta = (double)de;
                D.sqg_in = (double)((long double)d.R_in * dRof(el));
                D.sqg_out = (double)((long double)d.R_out * dRof(er));
            }
            D.tsqg = put(sqg);
            D.tef = put(ef);
            D.den_in *= D.sqg_in;
            D.den_out *= D.sqg_out;
        }
        if (precision == VLB_MIXED) {
            // FP32 path: populations scaled by 1/W (f/omega at the nodes, O(1) values); the
            // kernels become diag(1/w) K diag(w), the equilibrium bases lose their w factor
            // and the wall tables are divided by W.  Moments and n_w sums weight by W; the
            // residual weight becomes W.
            InstDesc& E = b->desc32[i];
            E = D;
            const int n1 = h.a1.nodes, n2 = h.a2.nodes;
            std::vector<double> K1s(h.a1.K), Kt2s(h.a2.Kt), B1s(h.a1.B), B2s(h.a2.B);
            for (int a = 0; a < n1; ++a)
                for (int c = 0; c < n1; ++c) K1s[a * n1 + c] *= h.a1.w[c] / h.a1.w[a];
            for (int a = 0; a < n2; ++a)
                for (int c = 0; c < n2; ++c) Kt2s[a * n2 + c] *= h.a2.w[c] / h.a2.w[a];
            for (int a = 0; a < n1; ++a)
                for (int l = 0; l <= h.a1.N; ++l) B1s[a * (h.a1.N + 1) + l] /= h.a1.w[a];
            for (int a = 0; a < n2; ++a)
                for (int l = 0; l <= h.a2.N; ++l) B2s[a * (h.a2.N + 1) + l] /= h.a2.w[a];
            std::vector<double> tins(tin), touts(tout);
            for (int k = 0; k < h.NV; ++k) { tins[k] *= invW[k]; touts[k] *= invW[k]; }
            E.tK1 = put(K1s); E.tKt2 = put(Kt2s);
            E.tB1 = put(B1s); E.tB2 = put(B2s);
            E.tfin = put(tins); E.tfout = put(touts);
            E.tWm = put(W);
            E.tresW = E.tWm;
        }
        if (precision == VLB_MIXED) b->desc32[i].offT = D.offT;
        offF += (size_t)2 * d.N_R * h.NV;
        offC += d.N_R;
    }
    b->state_n = offF;
    b->ncells = offC;

    // auxiliary-kernel work list: per instance and distribution, runs of <= kTileCells
    // cells, one per wavefront, padded to blocks of kWavesPerBlock wavefronts
    LaunchGroup g{0, 0, 0.0};
    for (int i = 0; i < B; ++i) {
        const InstDesc& D = b->desc[i];
        const int nruns = (D.NR + kTileCells - 1) / kTileCells;
        const int per = (D.NR + nruns - 1) / nruns;
        for (int dist = 0; dist < 2; ++dist) {
            int made = 0;
            for (int s = 0; s < D.NR; s += per) {
                b->work.push_back({i, dist, s, std::min(per, D.NR - s)});
                ++made;
            }
            while (made % kWavesPerBlock) { b->work.push_back({i, dist, 0, 0}); ++made; }
        }
        if (b->inst[i].wide) {   // scratch of the four-launch stage
            InstHost& h = b->inst[i];
            h.wY = b->wide_n; b->wide_n += (size_t)2 * D.NR * D.NV;
            h.wEq = b->wide_n; b->wide_n += (size_t)D.NR * kEqStride;
            h.wNw = b->wide_n; b->wide_n += (size_t)pad4(2 * wide_chunks(D.NV));
            h.wPart = b->wide_n; b->wide_n += wide_part_doubles(D.NR, D.NV);
            continue;
        }
        g.kmax = std::max({g.kmax, ktab_elems(D.Q1, D.Q2, 4), ktab_elems(D.Q1, D.Q2, 8)});
        g.pops += 2.0 * D.NR * D.NV;
    }
    g.kmax = pad4(g.kmax);
    if (stage_lds(g.kmax, sizeof(double)) > 160 * 1024) {
        delete b;
        return fail(VLB_EINVAL, "velocity sets too large for LDS (%zu bytes)", stage_lds(g.kmax, sizeof(double)));
    }
    b->groups.push_back(g);
    // stage-kernel block list: sized for the shortest cell run, built for the default
    build_blocks(b, kMinTile);
    b->max_blocks = b->blocks.size();
    build_blocks(b, kTileCells);

    vlb_status st = layout_and_alloc(b, defer_alloc == 0);
    if (st != VLB_OK) { delete b; return st; }
    if (!defer_alloc) {
        st = finish_setup(b);
        if (st != VLB_OK) { vlb_batch_destroy(b); return st; }
    }
    *out = b;
    return VLB_OK;
}

void vlb_batch_destroy(vlb_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (TimedLaunch& t : b->timed) { (void)hipEventDestroy(t.start); (void)hipEventDestroy(t.stop); }
    for (hipEvent_t e : b->event_pool) (void)hipEventDestroy(e);
    if (b->owns && b->ws) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipFree(b->ws);
    }
    delete b;
}

vlb_status vlb_batch_workspace_bytes(const vlb_batch* b, size_t* bytes) {
    if (!b || !bytes) return fail(VLB_EINVAL, "null argument");
    *bytes = b->total_bytes;
    return VLB_OK;
}

vlb_status vlb_batch_bind_workspace(vlb_batch* b, void* dev_ptr, size_t bytes) {
    if (!b || !dev_ptr) return fail(VLB_EINVAL, "null argument");
    if (((size_t)dev_ptr & 255) != 0) return fail(VLB_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < b->total_bytes) return fail(VLB_ENOMEM, "workspace of %zu bytes < required %zu", bytes, b->total_bytes);
    if (b->owns && b->ws) {
        HIP_TRY(hipStreamSynchronize(b->stream));
        HIP_TRY(hipFree(b->ws));
    }
    drop_graphs(b);   // captured kernels point into the old workspace
    b->ws = (char*)dev_ptr;
    b->owns = false;
    return finish_setup(b);
}

vlb_status vlb_batch_info(const vlb_batch* b, int inst, int* N_R, int* NV, int* nodes1, int* nodes2, double* dt,
                          size_t* state_offset) {
    if (!b || inst < 0 || inst >= b->B) return fail(VLB_EINVAL, "bad instance");
    const InstDesc& D = b->desc[inst];
    if (N_R) *N_R = D.NR;
    if (NV) *NV = D.NV;
    if (nodes1) *nodes1 = D.Q1;
    if (nodes2) *nodes2 = D.Q2;
    if (dt) *dt = D.dt;
    if (state_offset) *state_offset = (size_t)D.offF;
    return VLB_OK;
}

vlb_status vlb_batch_state_size(const vlb_batch* b, size_t* n) {
    if (!b || !n) return fail(VLB_EINVAL, "null argument");
    *n = b->state_n;
    return VLB_OK;
}

vlb_status vlb_batch_velocities(const vlb_batch* b, int inst, double* p1, double* w1, double* p2, double* w2) {
    if (!b || inst < 0 || inst >= b->B) return fail(VLB_EINVAL, "bad instance");
    const InstHost& h = b->inst[inst];
    if (p1) std::memcpy(p1, h.a1.p.data(), h.a1.p.size() * sizeof(double));
    if (w1) std::memcpy(w1, h.a1.w.data(), h.a1.w.size() * sizeof(double));
    if (p2) std::memcpy(p2, h.a2.p.data(), h.a2.p.size() * sizeof(double));
    if (w2) std::memcpy(w2, h.a2.w.data(), h.a2.w.size() * sizeof(double));
    return VLB_OK;
}

vlb_status vlb_set_wall(vlb_batch* b, int inst, int side, double u, double T) {
    if (!check_instance(b, inst) || (side != 0 && side != 1) || !(T > 0) || !std::isfinite(u))
        return fail(VLB_EINVAL, "bad wall arguments");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    InstHost& h = b->inst[inst];
    InstDesc& D = b->desc[inst];
    std::vector<double> tbl;
    double den = 0;
    wall_table(h, u, T, side, tbl, den);
    if (D.form == 1) den *= side == 0 ? D.sqg_in : D.sqg_out;   // f-tilde: ghosts carry sqrt(g_wall)
    const int off = side == 0 ? D.tfin : D.tfout;
    std::copy(tbl.begin(), tbl.end(), b->tab.begin() + D.offT + off);
    if (b->precision == VLB_MIXED) {
        const InstDesc& E = b->desc32[inst];
        const int off32 = side == 0 ? E.tfin : E.tfout;
        for (int k = 0; k < h.NV; ++k) b->tab[E.offT + off32 + k] = tbl[k] * b->tab[D.offT + D.tresW + k];
    }
    if (side == 0) { h.d.u_in = u; h.d.T_in = T; D.den_in = den; D.T_in = T; }
    else { h.d.u_out = u; h.d.T_out = T; D.den_out = den; D.T_out = T; }
    if (b->precision == VLB_MIXED) {
        InstDesc& E = b->desc32[inst];
        E.den_in = D.den_in; E.den_out = D.den_out; E.T_in = D.T_in; E.T_out = D.T_out;
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    return upload_tables(b);
}

vlb_status vlb_init_equilibrium(vlb_batch* b, int inst, const double* n, const double* u1, const double* u2,
                                const double* T) {
    if (!b || !n || !u1 || !u2 || !T || inst < -1 || inst >= b->B) return fail(VLB_EINVAL, "bad arguments");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    vlb_status es = ensure_precision(b, false);
    if (es != VLB_OK) return es;
    std::vector<double> host(b->state_n);
    HIP_TRY(hipMemcpyAsync(host.data(), b->F(0), b->state_n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    size_t cell = 0;
    for (int i = 0; i < b->B; ++i) {
        const int NR = b->desc[i].NR;
        if (inst == -1 || inst == i) {
            const size_t o = inst == -1 ? cell : 0;
            for (int s = 0; s < NR; ++s)
                if (!(n[o + s] > 0) || !(T[o + s] > 0) || !std::isfinite(u1[o + s]) || !std::isfinite(u2[o + s]))
                    return fail(VLB_EINVAL, "invalid equilibrium fields at instance %d cell %d", i, s);
            equilibrium_state(b->inst[i], n + o, u1 + o, u2 + o, T + o, host.data() + b->desc[i].offF);
        }
        cell += NR;
    }
    return set_state_device(b, host.data());
}

vlb_status vlb_set_state(vlb_batch* b, const double* host, size_t n) {
    if (!b || !host || n != b->state_n) return fail(VLB_EINVAL, "state size mismatch (%zu vs %zu)", n, b ? b->state_n : 0);
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    for (size_t x = 0; x < n; ++x)
        if (!std::isfinite(host[x])) return fail(VLB_ENONFINITE, "non-finite value at element %zu", x);
    return set_state_device(b, host);
}

vlb_status vlb_get_state(vlb_batch* b, double* host, size_t n) {
    if (!b || !host || n != b->state_n) return fail(VLB_EINVAL, "state size mismatch");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    vlb_status es = ensure_precision(b, false);
    if (es != VLB_OK) return es;
    HIP_TRY(hipMemcpyAsync(host, b->F(0), n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return VLB_OK;
}

vlb_status vlb_step(vlb_batch* b, long nsteps) {
    if (!b || nsteps < 0) return fail(VLB_EINVAL, "bad arguments");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    vlb_status s = ensure_precision(b, b->precision == VLB_MIXED);
    if (s != VLB_OK) return s;
    return step_current(b, nsteps);
}

vlb_status vlb_step_fp64(vlb_batch* b, long nsteps) {
    if (!b || nsteps < 0) return fail(VLB_EINVAL, "bad arguments");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    vlb_status s = ensure_precision(b, false);
    if (s != VLB_OK) return s;
    return step_current(b, nsteps);
}

vlb_status vlb_apply_L(vlb_batch* b, double* L, size_t n) {
    if (!b || !L || n != b->state_n) return fail(VLB_EINVAL, "size mismatch");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    vlb_status s = run_stage(b, 0, false, true);
    if (s != VLB_OK) return s;
    if (b->cur32) {
        // unscale the FP32 result into the FP64 scratch buffer (F * W on the device)
        const int nblocks = (int)(b->work.size() / kWavesPerBlock);
        HIP_TRY(launch_convert(kConvFrom32, nblocks, b->stream, b->ddesc32(), b->dwork(), b->dtab(), b->F(1), b->F32(1)));
    }
    HIP_TRY(hipMemcpyAsync(L, b->F(1), n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return VLB_OK;
}

vlb_status vlb_moments(vlb_batch* b, int inst, double* n, double* u1, double* u2, double* T, double* T12,
                       double* q1, double* q2) {
    if (!check_instance(b, inst)) return fail(VLB_EINVAL, "bad instance");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    vlb_status es = ensure_precision(b, false);
    if (es != VLB_OK) return es;
    const int nblocks = (int)(b->work.size() / kWavesPerBlock);
    HIP_TRY(launch_diag(nblocks, b->stream, b->ddesc(), b->dwork(), b->dtab(), b->F(0), b->diag()));
    const InstDesc& D = b->desc[inst];
    std::vector<double> h((size_t)D.NR * 7);
    HIP_TRY(hipMemcpyAsync(h.data(), b->diag() + (size_t)D.offC * 7, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    double* outs[7] = {n, u1, u2, T, T12, q1, q2};
    for (int q = 0; q < 7; ++q)
        if (outs[q])
            for (int s = 0; s < D.NR; ++s) outs[q][s] = h[(size_t)s * 7 + q];
    return VLB_OK;
}

vlb_status vlb_residual(vlb_batch* b, double* r) {
    if (!b || !r) return fail(VLB_EINVAL, "null argument");
    if (!b->have_resid) return fail(VLB_ESTATE, "no step recorded since the last state change");
    return read_residual(b, r);
}

vlb_status vlb_total_mass(vlb_batch* b, double* Ntot) {
    if (!b || !Ntot) return fail(VLB_EINVAL, "null argument");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    HIP_TRY(launch_reduce(b->B, b->stream, b->ddesc(), b->dtab(), b->rpart(), b->M(0), b->resid(), b->massv(), 0));
    HIP_TRY(hipMemcpyAsync(Ntot, b->massv(), b->B * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return VLB_OK;
}

static vlb_status run_to_steady_impl(vlb_batch* b, double tol, long max_steps, int check_every, long* steps,
                                     double* r);

vlb_status vlb_run_to_steady(vlb_batch* b, double tol, long max_steps, int check_every, long* steps, double* r) {
    const auto t0 = std::chrono::steady_clock::now();
    const vlb_status s = run_to_steady_impl(b, tol, max_steps, check_every, steps, r);
    if (b) b->run_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return s;
}

vlb_status vlb_batch_last_run_seconds(const vlb_batch* b, double* seconds) {
    if (!b || !seconds) return fail(VLB_EINVAL, "null argument");
    *seconds = b->run_seconds;
    return VLB_OK;
}

static vlb_status run_to_steady_impl(vlb_batch* b, double tol, long max_steps, int check_every, long* steps,
                                     double* r) {
    if (!b || !(tol > 0) || max_steps < 1 || check_every < 1) return fail(VLB_EINVAL, "bad arguments");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    std::vector<long> conv(b->B, -1);
    std::vector<double> res(b->B, INFINITY);
    long done = 0;
    vlb_status s = ensure_precision(b, false);
    if (s != VLB_OK) return s;
    const bool mixed = b->precision == VLB_MIXED;
    if (b->theta.size() != (size_t)b->B) reset_run_state(b, nullptr);
    if (b->warm.size() != (size_t)b->B) b->warm.assign(b->B, 0);
    if (b->fallback_at.size() != (size_t)b->B) b->fallback_at.assign(b->B, -1);
    if (b->best_res.size() != (size_t)b->B) b->best_res.assign(b->B, INFINITY);
    if (b->best_at.size() != (size_t)b->B) b->best_at.assign(b->B, 0);
    std::vector<double>& best = b->best_res;
    std::vector<long>& best_at = b->best_at;
    // converged instances retire: the stage kernels stop advancing them (their state,
    // moments and residual stay at the converged step); all are reinstated on return
    struct Reinstate {
        vlb_batch* b;
        bool dirty = false;
        ~Reinstate() {
            if (!dirty) return;
            b->active.clear();
            build_blocks(b, b->tile_set);
            (void)upload_blocks(b);
        }
    } guard{b};
    int remaining = b->B;
    while (done < max_steps && remaining > 0) {
        // FP64 steps: the plain solver's residual of the current iterate (mixed batches
        // take one, then check_every - 1 defect-correction steps in FP32)
        const bool dc = mixed;
        const long n = dc ? 1 : std::min<long>(check_every, max_steps - done);
        s = step_current(b, n);
        if (s != VLB_OK) return s;
        done += n;
        b->run_steps += n;
        s = read_residual(b, res.data());
        if (s != VLB_OK) return s;
        bool retired = false, dc_split = false;
        std::vector<int> restart(b->B, -1);
        bool any_restart = false;
        for (int i = 0; i < b->B; ++i) {
            if (conv[i] >= 0) continue;
            if (res[i] < tol) {
                conv[i] = done;
                --remaining;
                if (b->active.empty()) b->active.assign(b->B, 1);
                b->active[i] = 0;
                retired = guard.dirty = true;
                continue;
            }
            if (!b->warm[i]) continue;
            // a warm start whose residual has not set a new low (by 1 %) for stall_window
            // steps is judged stuck and restarted from the cold rest state
            if (res[i] < 0.99 * best[i]) {
                best[i] = res[i];
                best_at[i] = b->run_steps;
            } else if (b->run_steps - best_at[i] >= b->stall_window) {
                restart[i] = 0;
                any_restart = true;
                b->warm[i] = 0;
                b->fallback_at[i] = b->run_steps;
            }
        }
        if (any_restart) {
            s = init_from_surrogate(b, restart);
            if (s != VLB_OK) return s;
            for (int i = 0; i < b->B; ++i)
                if (restart[i] == 0) {   // the cold start is a new problem for the correction
                    b->theta[i] = 1.0;
                    b->dc_miss[i] = 0;
                    b->dc_hit[i] = 0;
                    b->dc_best[i] = INFINITY;
                    b->dc_best_at[i] = b->run_steps;
                    b->dc_hist[i].clear();
                    b->trial_at[i] = b->trial_end[i] = -1;
                    b->trial_gap[i] = 0;
                    b->dc64_at[i] = -1;
                    if (b->dc64[i]) {
                        b->dc64[i] = 0;
                        --b->n_dc64;
                        dc_split = true;
                    }
                }
        }
        if (dc) {
            // relaxation of the defect correction: an instance that sets no new residual low
            // (by 1 %) at three checks in a row has its update halved (a mode the linearised
            // operator overshoots otherwise makes the iteration cycle), one that sets eight
            // in a row has it doubled back towards the full correction.  The linearised
            // operator can also leave the correction converging far slower than FP64 steps
            // would: an instance whose update was just halved, or whose residual fell by
            // less than kSlowDecade over the last kRateChecks checks, is put on an FP64 trial
            // (kTrialChecks checks of FP64 steps, beside the others' FP32 steps; trials of
            // an instance kTrialGap trial lengths apart, twice as far after each lost one).
            // It keeps FP64 steps if their residual fell by kTrialDrop over the trial and
            // decayed kTrialGain times faster than the correction's over the checks before,
            // else it returns to the correction.  On FP64 steps an instance that sets no new
            // low for kDcStuck steps (plain stepping can settle into a cycle the relaxed
            // correction damps) returns to the correction at the smallest relaxation.
            const long trial_len = (long)kTrialChecks * check_every;
            auto set_fp64 = [&](int i, int on) {
                if (b->dc64[i] == on) return;
                b->dc64[i] = on;
                b->n_dc64 += on ? 1 : -1;
                dc_split = true;
            };
            auto back_to_dc = [&](int i) {
                set_fp64(i, 0);
                b->dc_hist[i].clear();
                b->dc_best[i] = res[i];
                b->dc_best_at[i] = b->run_steps;
                b->dc_miss[i] = b->dc_hit[i] = 0;
            };
            for (int i = 0; i < b->B; ++i) {
                if (conv[i] >= 0) continue;
                if (b->dc64_at[i] >= 0) {   // on FP64 steps after a won trial
                    if (res[i] < 0.99 * b->dc_best[i]) {
                        b->dc_best[i] = res[i];
                        b->dc_best_at[i] = b->run_steps;
                    } else if (b->run_steps - b->dc_best_at[i] >= kDcStuck) {
                        back_to_dc(i);
                        b->dc64_at[i] = -1;
                        b->theta[i] = 0.125;
                        b->trial_end[i] = b->run_steps;
                        b->trial_gap[i] *= 2;
                    }
                    continue;
                }
                if (b->trial_at[i] >= 0) {   // FP64 trial in progress
                    const long len = b->run_steps - b->trial_at[i];
                    if (len < trial_len) continue;
                    const double rate64 = std::log(b->trial_r0[i] / res[i]) / (double)len;
                    if (b->trial_r0[i] >= kTrialDrop * res[i] && rate64 > kTrialGain * std::max(b->dc_rate[i], 0.0)) {
                        b->dc64_at[i] = b->trial_at[i];
                        b->dc_best[i] = res[i];
                        b->dc_best_at[i] = b->run_steps;
                    } else {
                        back_to_dc(i);
                        b->trial_gap[i] *= 2;
                    }
                    b->trial_at[i] = -1;
                    b->trial_end[i] = b->run_steps;
                    continue;
                }
                auto& h = b->dc_hist[i];
                h.emplace_back(b->run_steps, res[i]);
                if (h.size() > (size_t)kRateChecks + 1) h.erase(h.begin());
                bool halved = false;
                if (res[i] < 0.99 * b->dc_best[i]) {
                    b->dc_best[i] = res[i];
                    b->dc_best_at[i] = b->run_steps;
                    b->dc_miss[i] = 0;
                    if (++b->dc_hit[i] >= 8) {
                        b->theta[i] = std::min(1.0, 2.0 * b->theta[i]);
                        b->dc_hit[i] = 0;
                    }
                } else {
                    b->dc_hit[i] = 0;
                    if (++b->dc_miss[i] >= 3) {
                        b->theta[i] = std::max(0.125, 0.5 * b->theta[i]);
                        b->dc_miss[i] = 0;
                        halved = true;
                    }
                }
                if (b->trial_gap[i] == 0) b->trial_gap[i] = kTrialGap * trial_len;
                const bool may_try = b->trial_end[i] < 0 || b->run_steps - b->trial_end[i] >= b->trial_gap[i];
                const bool slow = h.size() == (size_t)kRateChecks + 1 && h.front().second < kSlowDecade * h.back().second;
                if (may_try && h.size() > (size_t)kTrialChecks && (halved || slow)) {
                    b->dc_rate[i] = std::log(h.front().second / h.back().second) /
                                    (double)(h.back().first - h.front().first);
                    b->trial_at[i] = b->run_steps;
                    b->trial_r0[i] = res[i];
                    set_fp64(i, 1);
                }
            }
        }
        if (retired && remaining > 0) {
            active_tile(b);
            s = upload_blocks(b);
            if (s != VLB_OK) return s;
        }
        if (dc_split || (retired && b->n_dc64 > 0)) {
            HIP_TRY(hipMemcpyAsync(b->dmask(), b->dc64.data(), b->B * sizeof(int), hipMemcpyHostToDevice, b->stream));
            build_blocks(b, b->tile);
            s = upload_blocks(b);
            if (s != VLB_OK) return s;
            guard.dirty = true;
        }
        if (dc && remaining > 0 && done < max_steps) {
            const long m = std::min<long>(check_every - 1, max_steps - done);
            if (m > 0) {
                s = defect_correction(b, m);
                if (s != VLB_OK) return s;
                for (int i = 0; i < b->B; ++i)
                    if (conv[i] < 0 && !b->dc64[i]) b->fp32_inst[i] += m;
                done += m;
                b->run_steps += m;
                b->fp32_steps += m;
            }
        }
    }
    if (steps) std::copy(conv.begin(), conv.end(), steps);
    if (r) std::copy(res.begin(), res.end(), r);
    return remaining ? fail(VLB_ENOTCONV, "%d instance(s) above tol after %ld steps", remaining, done) : VLB_OK;
}

vlb_status vlb_mixed_report(const vlb_batch* b, double* theta, long* fp64_from, long* fp32_steps) {
    if (!b || (!theta && !fp64_from && !fp32_steps)) return fail(VLB_EINVAL, "null argument");
    const bool have = b->theta.size() == (size_t)b->B;
    for (int i = 0; i < b->B; ++i) {
        if (theta) theta[i] = have ? b->theta[i] : 1.0;
        if (fp64_from) fp64_from[i] = have ? b->dc64_at[i] : -1;
        if (fp32_steps) fp32_steps[i] = have ? b->fp32_inst[i] : 0;
    }
    return VLB_OK;
}

vlb_status vlb_mixed_fp32_steps(const vlb_batch* b, long* n) {
    if (!b || !n) return fail(VLB_EINVAL, "null argument");
    *n = b->fp32_steps;
    return VLB_OK;
}

vlb_status vlb_batch_set_tile(vlb_batch* b, int cells_per_run) {
    if (!b || cells_per_run < kMinTile || cells_per_run > kMaxTile) return fail(VLB_EINVAL, "tile out of range");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    HIP_TRY(hipStreamSynchronize(b->stream));
    build_blocks(b, cells_per_run);
    b->tile_set = cells_per_run;
    return upload_blocks(b);
}

vlb_status vlb_batch_get_tile(const vlb_batch* b, int* cells_per_run) {
    if (!b || !cells_per_run) return fail(VLB_EINVAL, "null argument");
    *cells_per_run = b->tile;
    return VLB_OK;
}

vlb_status vlb_batch_autotune(vlb_batch* b, int steps, int* chosen, double* ms_per_step) {
    if (!b || steps < 1) return fail(VLB_EINVAL, "bad arguments");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    // keep the state: the trial steps run on a copy and the original is put back
    const bool f32 = b->cur32;
    const size_t bytes = b->state_n * (f32 ? sizeof(float) : sizeof(double));
    void* keep = nullptr;
    HIP_TRY(hipMalloc(&keep, bytes));
    void* cur = f32 ? (void*)b->F32(0) : (void*)b->F(0);
    HIP_TRY(hipMemcpyAsync(keep, cur, bytes, hipMemcpyDeviceToDevice, b->stream));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const bool timing = b->timing;
    b->timing = false;
    int best = b->tile;
    float best_ms = 1e30f;
    vlb_status st = VLB_OK;
    // every length: the launch's block count against the 256 CUs (a last, nearly empty
    // round of blocks costs a whole block time), the halo reads and the per-block set-up
    // all move with it, not monotonically.  Each length keeps the best of kTuneReps timed
    // runs: a small instance's few-millisecond timings otherwise pick among neighbouring
    // lengths by noise.
    constexpr int kTuneReps = 3;
    for (int tile = kMinTile; tile <= kMaxTile && st == VLB_OK; ++tile) {
        build_blocks(b, tile);
        st = upload_blocks(b);
        if (st != VLB_OK) break;
        st = step_current(b, 1);   // warm-up (also captures nothing: single plain step)
        if (st != VLB_OK) break;
        for (int rep = 0; rep < kTuneReps; ++rep) {
            HIP_TRY(hipEventRecord(e0, b->stream));
            st = step_current(b, steps);
            if (st != VLB_OK) break;
            HIP_TRY(hipEventRecord(e1, b->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_ms) { best_ms = ms; best = tile; }
        }
    }
    b->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    build_blocks(b, best);
    b->tile_set = best;
    vlb_status s2 = upload_blocks(b);
    HIP_TRY(hipMemcpyAsync(cur, keep, bytes, hipMemcpyDeviceToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    (void)hipFree(keep);
    if (st != VLB_OK) return st;
    if (s2 != VLB_OK) return s2;
    b->have_resid = false;
    if (chosen) *chosen = best;
    if (ms_per_step) *ms_per_step = best_ms / steps;
    return refresh_moments(b);
}

vlb_status vlb_batch_set_persistent(vlb_batch* b, int max_blocks) {
    if (!b || max_blocks < 0) return fail(VLB_EINVAL, "bad arguments");
    b->persist_max = max_blocks;
    return VLB_OK;
}

vlb_status vlb_batch_set_graphs(vlb_batch* b, int enable) {
    if (!b) return fail(VLB_EINVAL, "null batch");
    b->use_graphs = enable != 0;
    return VLB_OK;
}

vlb_status vlb_timing_enable(vlb_batch* b, int enable) {
    if (!b) return fail(VLB_EINVAL, "null batch");
    b->timing = enable != 0;
    return VLB_OK;
}

vlb_status vlb_timing_query(vlb_batch* b, int max_groups, int* ngroups, int* bits, long* launches, double* total_ms,
                            double* alg_bytes) {
    if (!b || max_groups < 0 || !ngroups) return fail(VLB_EINVAL, "bad arguments");
    HIP_TRY(hipStreamSynchronize(b->stream));
    const int G = (int)b->groups.size() * 2;   // (group, precision)
    std::vector<long> n(G, 0);
    std::vector<double> ms(G, 0.0), by(G, 0.0);
    for (TimedLaunch& t : b->timed) {
        float e = 0.f;
        HIP_TRY(hipEventElapsedTime(&e, t.start, t.stop));
        const int key = t.group * 2 + (t.fp32 ? 1 : 0);
        n[key] += 1;
        ms[key] += e;
        by[key] += t.bytes;
        b->event_pool.push_back(t.start);
        b->event_pool.push_back(t.stop);
    }
    b->timed.clear();
    int out = 0;
    for (int g = 0; g < G; ++g) {
        if (n[g] == 0) continue;
        if (out < max_groups) {
            if (bits) bits[out] = (g & 1) ? 32 : 64;
            if (launches) launches[out] = n[g];
            if (total_ms) total_ms[out] = ms[g];
            if (alg_bytes) alg_bytes[out] = by[g];
        }
        ++out;
    }
    *ngroups = out;
    return VLB_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ learned warm start

namespace {

// The surrogate covers the Couette family it was trained on: inner wall moving, outer
// wall at rest, both at T_w = 1, tau = Kn sqrt(pi/8)/n.
bool surrogate_eligible(const vlb_couette_desc& d) {
    return d.T_in == 1.0 && d.T_out == 1.0 && d.u_out == 0.0 && d.u_in > 0.0 && d.tau_model == VLB_TAU_AOKI &&
           d.Kn > 0.0 && d.R_in > 0.0;
}

// Inputs of every cell: (log10 Kn, u_w, beta, rho) mapped affinely from the box
// [-2, 1] x [0.05, 0.5] x [0.3, 0.8] x [0, 1] to [-1, 1]^4.
void surrogate_features(const vlb_batch* b, float* X) {
    size_t c = 0;
    for (int i = 0; i < b->B; ++i) {
        const vlb_couette_desc& d = b->inst[i].d;
        const std::vector<double>& Rf = b->inst[i].Rf;
        const double f0 = (std::log10(d.Kn) + 0.5) / 1.5, f1 = (d.u_in - 0.275) / 0.225,
                     f2 = (d.R_in / d.R_out - 0.55) / 0.25;
        for (int s = 0; s < d.N_R; ++s, ++c) {
            const double rho = (0.5 * (Rf[s] + Rf[s + 1]) - d.R_in) / (d.R_out - d.R_in);
            X[4 * c] = (float)f0;
            X[4 * c + 1] = (float)f1;
            X[4 * c + 2] = (float)f2;
            X[4 * c + 3] = (float)(2.0 * rho - 1.0);
        }
    }
}

// Initial state of the instances from the surrogate outputs in sy(): use[i] = 1 warm,
// 0 the cold rest state, -1 left as it is; FP64 buffers.
vlb_status init_from_surrogate(vlb_batch* b, const std::vector<int>& use) {
    std::vector<double> par(2 * (size_t)b->B);
    for (int i = 0; i < b->B; ++i) {
        par[2 * i] = b->inst[i].d.u_in;
        par[2 * i + 1] = use[i] > 0 ? 1.0 : (use[i] == 0 ? 0.0 : -1.0);
    }
    HIP_TRY(hipMemcpyAsync(b->wpar(), par.data(), par.size() * sizeof(double), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(launch_warm_profile(b->B, b->stream, b->ddesc(), b->dtab(), b->sy(), b->wpar(), b->prof()));
    const int nblocks = (int)(b->work.size() / kWavesPerBlock);
    HIP_TRY(launch_init_profile(nblocks, b->stream, b->ddesc(), b->dwork(), b->dtab(), b->prof(), b->wpar(),
                                b->F(0)));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->cur32 = false;
    b->lin = false;
    b->have_resid = false;
    return refresh_moments(b);
}

}  // namespace

extern "C" {

vlb_status vlb_batch_surrogate_samples(vlb_batch* b, float* X, float* T, size_t ncells) {
    if (!b || !X || !T || ncells != b->ncells) return fail(VLB_EINVAL, "need arrays of %zu cells", b ? b->ncells : 0);
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    for (int i = 0; i < b->B; ++i)
        if (!surrogate_eligible(b->inst[i].d))
            return fail(VLB_EINVAL, "instance %d is outside the surrogate's Couette family", i);
    vlb_status es = ensure_precision(b, false);
    if (es != VLB_OK) return es;
    const int nblocks = (int)(b->work.size() / kWavesPerBlock);
    HIP_TRY(launch_diag(nblocks, b->stream, b->ddesc(), b->dwork(), b->dtab(), b->F(0), b->diag()));
    std::vector<double> h(b->ncells * 7);
    HIP_TRY(hipMemcpyAsync(h.data(), b->diag(), h.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    surrogate_features(b, X);
    size_t c = 0;
    for (int i = 0; i < b->B; ++i) {
        const double uw = b->inst[i].d.u_in;
        for (int s = 0; s < b->inst[i].d.N_R; ++s, ++c) {
            const double* o = &h[c * 7];
            T[4 * c] = (float)((o[0] - 1.0) * 10.0);
            T[4 * c + 1] = (float)(o[1] * 10.0);
            T[4 * c + 2] = (float)(o[2] / uw);
            T[4 * c + 3] = (float)((o[3] - 1.0) * 10.0);
        }
    }
    return VLB_OK;
}

vlb_status vlb_batch_warm_start(vlb_batch* b, vlb_mlp* m, int probe_steps, int* used_warm) {
    if (!b || !m || probe_steps < 0) return fail(VLB_EINVAL, "bad arguments");
    if (!b->ws) return fail(VLB_ESTATE, "no workspace bound");
    vlb_status s = ensure_precision(b, false);
    if (s != VLB_OK) return s;
    std::vector<float> X(b->ncells * 4);
    surrogate_features(b, X.data());
    std::vector<int> elig(b->B), use(b->B, 0);
    bool any = false;
    for (int i = 0; i < b->B; ++i) any |= (elig[i] = surrogate_eligible(b->inst[i].d) ? 1 : 0) != 0;
    HIP_TRY(hipMemcpyAsync(b->sfeat(), X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    HIP_TRY(hipStreamSynchronize(mlp_stream(m)));
    s = mlp_infer(m, b->sfeat(), (long)b->ncells, b->sy(), 1, b->stream);
    if (s != VLB_OK) return s;
    if (any && probe_steps > 0) {
        // the acceptance probe: the FP64 residual after probe_steps steps from each start
        std::vector<double> rc(b->B), rw(b->B);
        s = init_from_surrogate(b, use);
        if (s == VLB_OK) s = step_current(b, probe_steps);
        if (s == VLB_OK) s = read_residual(b, rc.data());
        if (s == VLB_OK) s = init_from_surrogate(b, elig);
        if (s == VLB_OK) s = step_current(b, probe_steps);
        if (s != VLB_OK) return s;
        // a warm start that diverges is rejected, not reported as an error
        HIP_TRY(hipMemcpyAsync(rw.data(), b->resid(), b->B * sizeof(double), hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
        for (int i = 0; i < b->B; ++i) use[i] = elig[i] && std::isfinite(rw[i]) && rw[i] < rc[i];
    } else {
        use = elig;
    }
    s = init_from_surrogate(b, use);
    if (s != VLB_OK) return s;
    reset_run_state(b, use.data());
    if (used_warm) std::copy(use.begin(), use.end(), used_warm);
    return VLB_OK;
}

vlb_status vlb_batch_set_stall_window(vlb_batch* b, long steps) {
    if (!b || steps < 1) return fail(VLB_EINVAL, "stall window must be >= 1 step");
    b->stall_window = steps;
    return VLB_OK;
}

vlb_status vlb_batch_warm_report(const vlb_batch* b, int* on_warm, long* fallback_at) {
    if (!b) return fail(VLB_EINVAL, "null batch");
    for (int i = 0; i < b->B; ++i) {
        if (on_warm) on_warm[i] = i < (int)b->warm.size() ? b->warm[i] : 0;
        if (fallback_at) fallback_at[i] = i < (int)b->fallback_at.size() ? b->fallback_at[i] : -1;
    }
    return VLB_OK;
}

}  // extern "C"

namespace vlb {
double force_operator_norm(const AxisTables& a1, const AxisTables& a2) { return force_norm(a1, a2); }
}  // namespace vlb

// ------------------------------------------------------------------ steps in caller scratch

namespace vlb {

// Host-side set-up of a batch that runs in caller-supplied device memory: velocity sets,
// grids, descriptors and block lists are built (host memory only, no HIP call) and the
// device bytes it needs, with the state kept in the caller's array, are returned.
vlb_status couette_noalloc_plan(int B, const vlb_couette_desc* descs, vlb_batch** out, size_t* bytes) {
    vlb_status st = vlb_batch_create_couette(out, B, descs, VLB_FP64, nullptr, 1);
    if (st != VLB_OK) return st;
    vlb_batch* b = *out;
    st = layout_and_alloc(b, false, true);
    if (st != VLB_OK) { vlb_batch_destroy(b); *out = nullptr; return st; }
    b->use_graphs = false;
    b->persist_max = 0;
    *bytes = b->total_bytes;
    return VLB_OK;
}

// nsteps RK3 steps of a planned batch on the caller's FP64 state F (device, the layout of
// vlb_get_state) with every other device buffer in scratch (>= the planned bytes,
// 256-byte aligned); resid (host, B entries, may be NULL) receives the residual of the
// last step.  Every scratch byte a kernel reads is written earlier in the same call.
// Synchronises the stream before returning.
vlb_status couette_noalloc_run(vlb_batch* b, double* F, long nsteps, double* resid, hipStream_t stream,
                               char* scratch) {
    b->stream = stream;
    b->ws = scratch;
    b->owns = false;
    b->ext_F0 = F;
    vlb_status st = upload_tables(b);
    if (st == VLB_OK) {
        hipError_t e = hipMemcpyAsync(b->dwork(), b->work.data(), b->work.size() * sizeof(WorkItem),
                                      hipMemcpyHostToDevice, b->stream);
        if (e != hipSuccess) st = fail(VLB_EDEVICE, "work list upload failed: %s", hipGetErrorString(e));
    }
    if (st == VLB_OK) st = upload_blocks(b);
    if (st == VLB_OK) st = refresh_moments(b);
    if (st == VLB_OK) st = step_current(b, nsteps);
    if (st == VLB_OK && resid) st = read_residual(b, resid);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (st == VLB_OK && e != hipSuccess) st = fail(VLB_EDEVICE, "stream synchronisation failed: %s", hipGetErrorString(e));
    return st;
}

}  // namespace vlb
