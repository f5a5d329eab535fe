// Host side of the expanding-channel path: channel geometry and connection
// coefficients (Sec. VI.A), velocity-set tables, dt limits, device buffers and the RK3
// driver of the channel stage kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "channel_internal.h"
#include "mlp_internal.h"
#include "vlb_internal.h"

using namespace vlb;

struct vlb_channel {
    int B = 0;
    hipStream_t stream = nullptr;
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;                  // private stream used only to capture step graphs
    hipGraphExec_t graph[2] = {nullptr, nullptr};      // [FP32 state]: kChanGraphSteps steps, no residual
    std::vector<vlb_channel_desc> d;
    std::vector<ChanDesc> desc;
    std::vector<double> tab;
    std::vector<long long> cbase;   // first cell of each instance
    // stage launches: one per velocity-tile class (T1, T2), its instances and block offsets
    struct Group {
        int T1, T2;
        std::vector<int> ilist;
        std::vector<long long> base, bbase;   // blocks of the interior and of the edge-band launch
        size_t off_ilist, off_base, off_bbase;
    };
    std::vector<Group> groups;
    // instances of the population kernel, [0] vielbein and [1] Cartesian split: one launch
    // each, a block per cell
    std::vector<int> pop_ilist[2];
    std::vector<long long> pop_base[2] = {{0}, {0}};
    size_t off_pop_ilist[2] = {0, 0}, off_pop_base[2] = {0, 0};
    size_t state_n = 0, ncells = 0;
    int threads = 64;
    int precision = VLB_FP64;
    std::vector<ChanDesc> desc32;   // FP32 descriptors (rescaled tables), mixed precision only
    bool cur32 = false;             // the current state lives in the FP32 buffers
    bool polishing = false;         // the last run_to_steady ended in FP64, state untouched since
    long fp32_steps = 0;            // steps of the FP32 phase of the last run_to_steady
    char* ws = nullptr;
    size_t off_F[3], off_F32[3], off_rpart, off_resid, off_diag, off_tab, off_desc, off_desc32, off_cbase,
        off_sbase, off_fld, total;
    size_t fld_n = 0;               // doubles of the largest instance's flow diagnostics
    bool have_resid = false;
    bool owns = false;              // ws allocated by the library (else bound by the caller)
    double run_seconds = 0.0;       // wall clock of the last vlb_channel_run_to_steady

    double* F(int i) { return (double*)(ws + off_F[i]); }
    float* F32(int i) { return (float*)(ws + off_F32[i]); }
    ChanDesc* ddesc32() { return (ChanDesc*)(ws + off_desc32); }
    long long* dsbase() { return (long long*)(ws + off_sbase); }
    double* rpart() { return (double*)(ws + off_rpart); }
    double* resid() { return (double*)(ws + off_resid); }
    double* diag() { return (double*)(ws + off_diag); }
    double* fld() { return (double*)(ws + off_fld); }
    double* dtab() { return (double*)(ws + off_tab); }
    ChanDesc* ddesc() { return (ChanDesc*)(ws + off_desc); }
    const int* gilist(const Group& g) { return (const int*)(ws + g.off_ilist); }
    const long long* gbase(const Group& g) { return (const long long*)(ws + g.off_base); }
    const long long* gbbase(const Group& g) { return (const long long*)(ws + g.off_bbase); }
    long long* dcbase() { return (long long*)(ws + off_cbase); }
};

namespace {

bool axis_ok(const vlb_axis& a) {
    return (a.kind == 0 || a.kind == 1) && a.Q >= 1 && a.Q <= kMaxQ && a.N >= 0 && a.N < a.Q && a.N <= kMaxN;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Wall of the expanding channel: 1 + phi(xi) = 1 + (r - 1)(1 + tanh(4 xi / L - 2)) / 2,
// phi' = (r - 1)(2 / L) sech^2(4 xi / L - 2), and chi(xi) = xi + (r - 1)(xi + (L/4) ln cosh(4 xi / L - 2)) / 2
// with d chi = (1 + phi) d xi (Eq. chi_canalie), in long double.
struct Wall {
    long double r, L;
    long double phi(long double x) const { return (r - 1) * (1 + std::tanh(4 * x / L - 2)) / 2; }
    long double dphi(long double x) const {
        const long double c = std::cosh(4 * x / L - 2);
        return (r - 1) * 2 / L / (c * c);
    }
    long double chi(long double x) const {
        const long double z = std::fabs(4 * x / L - 2);
        const long double lncosh = z + std::log1p(std::exp(-2 * z)) - std::log(2.0L);
        return x + (r - 1) * (x + L / 4 * lncosh) / 2;
    }
};

// Move the current state between the FP64 buffer and the scaled FP32 buffer.
vlb_status channel_precision(vlb_channel* c, bool want32) {
    if (c->cur32 == want32) return VLB_OK;
    if (want32 && c->precision != VLB_MIXED) return set_error(VLB_ESTATE, "channel batch has no FP32 buffers");
    VLB_HIP_TRY(launch_channel_convert(want32 ? 1 : 0, (long long)c->state_n, c->stream,
                                       c->precision == VLB_MIXED ? c->ddesc32() : c->ddesc(), c->dsbase(), c->B,
                                       c->dtab(), c->F(0), c->F32(0)));
    c->cur32 = want32;
    return VLB_OK;
}

}  // namespace

extern "C" {

namespace {
vlb_status channel_device_setup(vlb_channel* c);
vlb_status channel_build(vlb_channel** out, int B, const vlb_channel_desc* descs, int precision, void* hip_stream,
                         bool alloc);
}  // namespace

vlb_status vlb_channel_create(vlb_channel** out, int B, const vlb_channel_desc* descs, int precision,
                              void* hip_stream) {
    return channel_build(out, B, descs, precision, hip_stream, true);
}

vlb_status vlb_channel_create_deferred(vlb_channel** out, int B, const vlb_channel_desc* descs, int precision,
                                       void* hip_stream) {
    return channel_build(out, B, descs, precision, hip_stream, false);
}

vlb_status vlb_channel_workspace_bytes(const vlb_channel* c, size_t* bytes) {
    if (!c || !bytes) return set_error(VLB_EINVAL, "null argument");
    *bytes = c->total;
    return VLB_OK;
}

vlb_status vlb_channel_bind_workspace(vlb_channel* c, void* dev_ptr, size_t bytes) {
    if (!c || !dev_ptr) return set_error(VLB_EINVAL, "null argument");
    if (c->ws) return set_error(VLB_ESTATE, "a workspace is already bound");
    if (bytes < c->total) return set_error(VLB_ENOMEM, "workspace of %zu bytes, need %zu", bytes, c->total);
    if ((uintptr_t)dev_ptr & 255) return set_error(VLB_EINVAL, "workspace must be 256-byte aligned");
    c->ws = (char*)dev_ptr;
    c->owns = false;
    vlb_status s = channel_device_setup(c);
    if (s != VLB_OK) c->ws = nullptr;
    return s;
}

namespace {
vlb_status channel_build(vlb_channel** out, int B, const vlb_channel_desc* descs, int precision, void* hip_stream,
                         bool alloc) {
    if (!out || B < 1 || !descs) return set_error(VLB_EINVAL, "need out, B >= 1 and descriptors");
    *out = nullptr;
    if (precision != VLB_FP64 && precision != VLB_MIXED) return set_error(VLB_EINVAL, "unsupported precision %d", precision);
    vlb_channel* c = new (std::nothrow) vlb_channel;
    if (!c) return set_error(VLB_ENOMEM, "host allocation failed");
    c->B = B;
    c->stream = (hipStream_t)hip_stream;
    c->d.assign(descs, descs + B);
    c->desc.resize(B);
    c->precision = precision;
    if (precision == VLB_MIXED) c->desc32.resize(B);
    std::map<std::tuple<int, int, int>, AxisTables> cache;
    auto get_axis = [&](const vlb_axis& a) -> const AxisTables* {
        auto key = std::make_tuple(a.kind, a.Q, a.N);
        auto it = cache.find(key);
        if (it == cache.end()) {
            AxisTables t;
            if (!build_axis(a.kind, a.Q, a.N, t)) return nullptr;
            it = cache.emplace(key, std::move(t)).first;
        }
        return &it->second;
    };
    size_t offF = 0, offC = 0;
    long long cells = 0;
    for (int i = 0; i < B; ++i) {
        const vlb_channel_desc& d = descs[i];
        if (!(d.N_lambda >= (d.half ? 3 : 6) && (d.half == 0 || d.half == 1) && (d.ends == 0 || d.ends == 1) &&
              std::isfinite(d.Q0) && d.N_xi >= 3 && d.xi_out > d.xi_in && d.r > 0 && d.L > 0 && d.Kn > 0 &&
              d.tau_model >= 0 && d.tau_model <= 2 && axis_ok(d.ax1) && d.ax1.kind == 1 && axis_ok(d.ax2) &&
              d.A >= 0 && d.A < 1 &&
              d.dt >= 0 && (d.dt > 0 || d.cfl > 0) && d.n_in > 0 && d.n_out > 0 && d.T_w > 0 && d.weno_eps >= 0 &&
              std::isfinite(d.weno_eps))) {
            delete c;
            return set_error(VLB_EINVAL, "invalid channel descriptor for instance %d (ax1 must be half range)", i);
        }
        if (d.cartesian != 0 && (d.cartesian != 1 || precision != VLB_FP64)) {
            delete c;
            return set_error(VLB_EINVAL, "instance %d: the Cartesian-split channel runs in FP64", i);
        }
        if (d.kernel < 0 || d.kernel > 2 || (d.kernel == 2 && precision != VLB_FP64)) {
            delete c;
            return set_error(VLB_EINVAL, "instance %d: kernel %d (0 auto, 1 velocity tiles, 2 population; the "
                             "population kernel runs in FP64)", i, d.kernel);
        }
        const AxisTables* a1 = get_axis(d.ax1);
        const AxisTables* a2 = get_axis(d.ax2);
        if (!a1 || !a2) {
            delete c;
            return set_error(VLB_EINVAL, "instance %d: velocity set construction failed", i);
        }
        const int n1 = a1->nodes, n2 = a2->nodes, NV = n1 * n2, NL = d.N_lambda, NX = d.N_xi;
        // velocity tiles of 16 x 16: at most two along one axis, not both.  The population
        // kernel (a block per cell, a thread per velocity) takes the Cartesian split, FP64
        // sets that need more tiles, and any FP64 set on request (measured slower than the
        // tiles wherever both apply: at 40..160 velocities most of its 256 threads idle)
        const int T1 = (n1 + 15) / 16, T2 = (n2 + 15) / 16;
        const bool tiles_ok = T1 * T2 <= 2;
        const bool pop = d.cartesian || d.kernel == 2 || (d.kernel == 0 && precision == VLB_FP64 && !tiles_ok);
        if (pop ? NV > kMaxNV : !tiles_ok) {
            delete c;
            return set_error(VLB_EINVAL,
                             "instance %d: %d x %d velocities exceed the kernel limits (16-node tiles: 1 x 1, 2 x 1 "
                             "or 1 x 2)", i, n1, n2);
        }
        ChanDesc& D = c->desc[i];
        D = ChanDesc{};
        D.NL = NL; D.NX = NX; D.Q1 = n1; D.Q2 = n2; D.NV = NV;
        D.kind1 = a1->kind; D.kind2 = a2->kind; D.N1 = a1->N; D.N2 = a2->N; D.Qh1 = a1->Q; D.Qh2 = a2->Q;
        D.tau_model = d.tau_model;
        D.Kn = d.Kn;
        D.weno_eps = d.weno_eps;
        D.half = d.half;
        D.ends = d.ends;
        D.cartesian = d.cartesian;
        D.offF = (long long)offF;
        D.offC = (long long)offC;
        D.offT = (long long)c->tab.size();
        auto put = [&](const std::vector<double>& v) {
            const int o = (int)(c->tab.size() - D.offT);
            c->tab.insert(c->tab.end(), v.begin(), v.end());
            return o;
        };
        D.tp1 = put(a1->p); D.tp2 = put(a2->p);
        D.tK1 = put(a1->K); D.tKt1 = put(a1->Kt); D.tK2 = put(a2->K); D.tKt2 = put(a2->Kt);
        D.tB1 = put(a1->B); D.tB2 = put(a2->B); D.tC1 = put(a1->C); D.tC2 = put(a2->C);
        D.tisf1 = put(a1->invsqrtfact); D.tisf2 = put(a2->invsqrtfact);
        // Maxwellians at rest with T_w: wall (n = 1), inlet, outlet reservoirs; [f' | f'']
        std::vector<double> g1(n1), g2(n2), fw(2 * NV), fin(2 * NV), fout(2 * NV), iW(NV), Wk(NV);
        axis_equilibrium_host(*a1, 0.0, d.T_w, g1.data());
        axis_equilibrium_host(*a2, 0.0, d.T_w, g2.data());
        double den_lo = 0.0, den_hi = 0.0;
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n2; ++b) {
                const int k = a * n2 + b;
                fw[k] = g1[a] * g2[b];
                fw[NV + k] = d.T_w * fw[k];
                if (a1->p[a] > 0) den_lo += a1->p[a] * fw[k];
                if (a1->p[a] < 0) den_hi += a1->p[a] * fw[k];
                Wk[k] = a1->w[a] * a2->w[b];
                iW[k] = 1.0 / Wk[k];
            }
        for (int k = 0; k < 2 * NV; ++k) { fin[k] = d.n_in * fw[k]; fout[k] = d.n_out * fw[k]; }
        D.den_lo = den_lo;
        D.den_hi = den_hi;
        D.tfw = put(fw); D.tfin = put(fin); D.tfout = put(fout); D.tiW = put(iW); D.tWm = put(Wk);
        if (precision == VLB_MIXED) {
            // FP32 path: populations scaled by 1/W_k (O(1) values); the kernels become
            // diag(1/w) K diag(w), the equilibrium bases lose their w factor, the ghost
            // Maxwellians are divided by W_k and the residual weight becomes W_k
            ChanDesc& E = c->desc32[i];
            E = D;
            std::vector<double> K1s(a1->K), Kt1s(a1->Kt), K2s(a2->K), Kt2s(a2->Kt), B1s(a1->B), B2s(a2->B);
            for (int a = 0; a < n1; ++a)
                for (int b = 0; b < n1; ++b) {
                    K1s[a * n1 + b] *= a1->w[b] / a1->w[a];
                    Kt1s[a * n1 + b] *= a1->w[b] / a1->w[a];
                }
            for (int a = 0; a < n2; ++a)
                for (int b = 0; b < n2; ++b) {
                    K2s[a * n2 + b] *= a2->w[b] / a2->w[a];
                    Kt2s[a * n2 + b] *= a2->w[b] / a2->w[a];
                }
            for (int a = 0; a < n1; ++a)
                for (int l = 0; l <= a1->N; ++l) B1s[a * (a1->N + 1) + l] /= a1->w[a];
            for (int a = 0; a < n2; ++a)
                for (int l = 0; l <= a2->N; ++l) B2s[a * (a2->N + 1) + l] /= a2->w[a];
            std::vector<double> fws(fw), fins(fin), fouts(fout);
            for (int k = 0; k < 2 * NV; ++k) {
                fws[k] *= iW[k % NV];
                fins[k] *= iW[k % NV];
                fouts[k] *= iW[k % NV];
            }
            E.tK1 = put(K1s); E.tKt1 = put(Kt1s); E.tK2 = put(K2s); E.tKt2 = put(Kt2s);
            E.tB1 = put(B1s); E.tB2 = put(B2s);
            E.tfw = put(fws); E.tfin = put(fins); E.tfout = put(fouts);
            E.tiW = D.tWm;
        }
        // geometry (Sec. VI.A): lambda in [-1, 1] (the upper half [0, 1] with a specular
        // centreline) and xi on equal cells
        const Wall w{(long double)d.r, (long double)d.L};
        std::vector<long double> lf(NL + 1), xf(NX + 1);
        // lambda faces: equal cells, or equal cells in eta with lambda = tanh(eta) / A
        // (Eq. canalie_stretch with H / 2 = 1; eta from 0 (half channel) or -artanh A to artanh A)
        for (int s = 0; s <= NL; ++s) {
            const long double t = d.half ? (long double)s / NL : -1.0L + 2.0L * s / NL;   // in [0, 1] or [-1, 1]
            lf[s] = d.A > 0 ? std::tanh(t * std::atanh((long double)d.A)) / (long double)d.A : t;
        }
        lf[0] = d.half ? 0.0L : -1.0L;   // the walls (and the centreline) exactly
        lf[NL] = 1.0L;
        for (int p = 0; p <= NX; ++p) xf[p] = (long double)d.xi_in + ((long double)d.xi_out - d.xi_in) * p / NX;
        std::vector<double> al(NX * NL), ar(NX * NL), glxx(NX * NL), glxl(NX * NL), xc((NX + 1) * NL),
            xa((NX + 1) * NL), dlam(NL), dchi(NX), vol(NX * NL);
        double vmax = 0.0, fmax1 = 0.0, fmax2 = 0.0;
        double pl_abs = 0.0, px_abs = 0.0;
        for (double v : a1->p) pl_abs = std::max(pl_abs, std::fabs(v));
        for (double v : a2->p) px_abs = std::max(px_abs, std::fabs(v));
        for (int s = 0; s < NL; ++s) dlam[s] = (double)(lf[s + 1] - lf[s]);
        for (int p = 0; p < NX; ++p) dchi[p] = (double)(w.chi(xf[p + 1]) - w.chi(xf[p]));
        for (int f = 0; f <= NX; ++f)
            for (int s = 0; s < NL; ++s) {
                const long double lam = (lf[s] + lf[s + 1]) / 2, a = lam * w.dphi(xf[f]);
                xa[f * NL + s] = (double)a;
                xc[f * NL + s] = (double)((1 + w.phi(xf[f])) / std::sqrt(1 + a * a));
            }
        for (int p = 0; p < NX; ++p) {
            const long double xcen = (xf[p] + xf[p + 1]) / 2, ph = w.phi(xcen), dph = w.dphi(xcen);
            for (int s = 0; s < NL; ++s) {
                const int cidx = p * NL + s;
                const long double lam = (lf[s] + lf[s + 1]) / 2;
                const long double sl = std::sqrt(1 + lf[s] * lf[s] * dph * dph);
                const long double sr = std::sqrt(1 + lf[s + 1] * lf[s + 1] * dph * dph);
                al[cidx] = (double)(sl / (1 + ph));
                ar[cidx] = (double)(sr / (1 + ph));
                // connection coefficients, discretised so that a uniform Maxwellian is exact
                const long double ql = xc[p * NL + s], qr = xc[(p + 1) * NL + s];
                glxl[cidx] = (double)((qr - ql) / dchi[p]);
                glxx[cidx] = (double)(-(sr - sl) / ((long double)dlam[s] * (1 + ph)) +
                                      lam / dchi[p] * (w.dphi(xf[p + 1]) * qr - w.dphi(xf[p]) * ql));
                vol[cidx] = dchi[p] * dlam[s];
                // advective rate bound of the cell: |V^lambda| / dlambda + |V^xi| / dchi
                double vx = 0.0;
                for (int e = 0; e < 2; ++e) {
                    const double cc = xc[(p + e) * NL + s], aa = xa[(p + e) * NL + s];
                    vx = std::max(vx, cc * (px_abs + std::fabs(aa) * pl_abs));
                }
                vmax = std::max(vmax, std::max(al[cidx], ar[cidx]) * pl_abs / dlam[s] + vx / dchi[p]);
                fmax1 = std::max(fmax1, std::fabs(glxx[cidx]));
                fmax2 = std::max(fmax2, std::fabs(glxl[cidx]));
            }
        }
        D.tal = put(al); D.tar = put(ar); D.tglxx = put(glxx); D.tglxl = put(glxl);
        D.txc = put(xc); D.txa = put(xa); D.tdlam = put(dlam); D.tdchi = put(dchi); D.tvol = put(vol);
        {   // flow diagnostics: phi, phi', xi at the cell centres, lambda faces and centres
            std::vector<double> geo((size_t)3 * NX + 2 * NL + 1);
            for (int p = 0; p < NX; ++p) {
                const long double xcen = (xf[p] + xf[p + 1]) / 2;
                geo[p] = (double)w.phi(xcen);
                geo[NX + p] = (double)w.dphi(xcen);
                geo[2 * NX + p] = (double)xcen;
            }
            for (int s = 0; s <= NL; ++s) geo[3 * NX + s] = (double)lf[s];
            for (int s = 0; s < NL; ++s) geo[3 * NX + NL + 1 + s] = (double)((lf[s] + lf[s + 1]) / 2);
            D.tgeo = put(geo);
        }
        double vclb = 0.0;   // Cartesian split: advective rate bound |V^lambda| / dlambda + |V^xi| / dchi
        if (d.cartesian) {
            // discrete metric a_p = (1 + phi_p)(phi_{p+1/2} - phi_{p-1/2}) / dchi_p (free-stream
            // preserving) and phi at the xi faces
            std::vector<double> clb(2 * (size_t)NX + 1);
            for (int p = 0; p < NX; ++p) {
                const long double xcen = (xf[p] + xf[p + 1]) / 2;
                clb[p] = (double)((1 + w.phi(xcen)) * (w.phi(xf[p + 1]) - w.phi(xf[p])) / (long double)dchi[p]);
            }
            for (int f = 0; f <= NX; ++f) clb[NX + f] = (double)w.phi(xf[f]);
            for (int p = 0; p < NX; ++p) {
                const double opf = 1.0 + (double)w.phi((xf[p] + xf[p + 1]) / 2);
                for (int s2 = 0; s2 < NL; ++s2)
                    for (int ia = 0; ia < n1; ++ia)
                        for (int jb = 0; jb < n2; ++jb) {
                            double vl = 0.0;
                            for (int e = 0; e < 2; ++e)
                                vl = std::max(vl, std::fabs(a1->p[ia] - (double)lf[s2 + e] * clb[p] * a2->p[jb]) / opf);
                            const double vx = std::max(1.0 + clb[NX + p], 1.0 + clb[NX + p + 1]) * std::fabs(a2->p[jb]);
                            vclb = std::max(vclb, vl / dlam[s2] + vx / dchi[p]);
                        }
            }
            D.tclb = put(clb);
        }
        D.ipf_in = (double)(1 / (1 + w.phi(xf[0])));
        D.ipf_out = (double)(1 / (1 + w.phi(xf[NX])));
        if (d.ends == 1) {
            // flow-rate ends (Sec. VI.C.1-2): per end and lambda row the prescribed flow rate
            // Q(lambda_s) = 3 Q0 / (H (1 + phi)) (1 - 4 lambda_s^2 / H^2), H = 2, the unit-density
            // Maxwellian of the Cartesian velocity (0, Q) in the face's triad (a = lambda phi',
            // c = 1 / sqrt(1 + a^2): u^lambda = -a c Q, u^xi = c Q), and its entering flow
            std::vector<double> Qrow(2 * NL), den(2 * NL), frow((size_t)2 * NL * 2 * NV), gl(n1), gx(n2);
            for (int e = 0; e < 2; ++e) {
                const int f = e ? NX : 0;
                for (int s = 0; s < NL; ++s) {
                    // the Cartesian split takes the profile velocity (0, Q) as it is (a = 0)
                    const long double lam = (lf[s] + lf[s + 1]) / 2, a = d.cartesian ? 0 : lam * w.dphi(xf[f]);
                    const long double cc = 1 / std::sqrt(1 + a * a);
                    const double Q = (double)(3 * (long double)d.Q0 / (2 * (1 + w.phi(xf[f]))) * (1 - lam * lam));
                    axis_equilibrium_host(*a1, (double)(-a * cc * Q), d.T_w, gl.data());
                    axis_equilibrium_host(*a2, (double)(cc * Q), d.T_w, gx.data());
                    double dd = 0.0;
                    for (int ia = 0; ia < n1; ++ia)
                        for (int jb = 0; jb < n2; ++jb) {
                            const int k = ia * n2 + jb;
                            const double fe = gl[ia] * gx[jb];
                            frow[((size_t)(e * NL + s) * 2) * NV + k] = fe;
                            frow[((size_t)(e * NL + s) * 2 + 1) * NV + k] = d.T_w * fe;
                            const double py = (double)(cc * (a2->p[jb] - a * a1->p[ia]));
                            if (e == 0 ? py > 0 : py < 0) dd += fe * py;
                        }
                    Qrow[e * NL + s] = Q;
                    den[e * NL + s] = dd;
                }
            }
            D.tQrow = put(Qrow); D.tden = put(den); D.tfrow = put(frow);
            if (precision == VLB_MIXED) {
                for (size_t x = 0; x < frow.size(); ++x) frow[x] *= iW[x % NV];
                c->desc32[i].tfrow = put(frow);
            }
        }
        if (precision == VLB_MIXED) {
            ChanDesc& E = c->desc32[i];
            E.tal = D.tal; E.tar = D.tar; E.tglxx = D.tglxx; E.tglxl = D.tglxl;
            E.txc = D.txc; E.txa = D.txa; E.tdlam = D.tdlam; E.tdchi = D.tdchi; E.tvol = D.tvol;
            E.ipf_in = D.ipf_in; E.ipf_out = D.ipf_out; E.tQrow = D.tQrow; E.tden = D.tden;
        }
        // dt: advection CFL combined with the force limit |lambda dt| <= sqrt(3) of RK3, capped
        // at 2 tau of the rest state (as for the Couette instances)
        const double rho =
            d.cartesian ? 0.0 : fmax1 * force_operator_norm(*a1, *a2) + fmax2 * force_operator_norm(*a2, *a1);
        const double inv1 = d.cartesian ? vclb : vmax + rho / std::sqrt(3.0);
        const double tau0 = d.tau_model == 0 ? d.Kn * 0.62665706865775012 : d.Kn;
        double dt = d.dt;
        if (dt == 0.0) {
            dt = std::min(d.cfl / inv1, 2.0 * tau0);
        } else if (dt > 1.0 / inv1 || dt > 2.5 * tau0) {
            delete c;
            return set_error(VLB_EUNSTABLE, "instance %d: dt=%g exceeds the stability limit %g", i, dt, 1.0 / inv1);
        }
        D.dt = dt;
        if (pop) {
            const int fm = d.cartesian ? 1 : 0;
            c->pop_ilist[fm].push_back(i);
            c->pop_base[fm].push_back(c->pop_base[fm].back() + (long long)NX * NL);
        } else {
            auto it = std::find_if(c->groups.begin(), c->groups.end(),
                                   [&](const vlb_channel::Group& g) { return g.T1 == T1 && g.T2 == T2; });
            if (it == c->groups.end()) {
                c->groups.push_back(vlb_channel::Group{T1, T2, {}, {0}, {0}, 0, 0, 0});
                it = c->groups.end() - 1;
            }
            // the stage kernel addresses an interior cell's stencil (seven xi columns) as one
            // buffer with 32-bit byte offsets
            if ((unsigned long long)7 * NL * NV * sizeof(double) >= (1ULL << 32)) {
                delete c;
                return set_error(VLB_EINVAL, "instance %d: N_lambda x velocities = %lld too large for the stage kernel",
                                 i, (long long)NL * NV);
            }
            // interior cells (3 <= s < NL - 3, 3 <= p < NX - 3) in lambda strips of up to
            // kChanStrip cells (a multiple of kChanWaves); edge-band cells in order
            const int NLi = std::max(NL - 6, 0), NXi = std::max(NX - 6, 0);
            D.strip = std::max(kChanWaves, std::min(kChanStrip, (NLi + kChanWaves - 1) / kChanWaves * kChanWaves));
            const long long nstrips = (NLi + D.strip - 1) / D.strip;
            const long long bcells = (long long)std::min(NL, 6) * NX + (long long)NLi * std::min(NX, 6);
            it->ilist.push_back(i);
            it->base.push_back(it->base.back() + (NXi > 0 ? nstrips * NXi * (D.strip / kChanWaves) : 0));
            it->bbase.push_back(it->bbase.back() + (bcells + kChanWaves - 1) / kChanWaves);
        }
        if (precision == VLB_MIXED) {   // fields set after the table section
            ChanDesc& E = c->desc32[i];
            E.dt = D.dt;
            E.strip = D.strip;
        }
        c->cbase.push_back(cells);
        c->fld_n = std::max(c->fld_n, (size_t)4 * NX * NL + (size_t)NX * (NL + 1) + 2 * (size_t)NX);
        cells += (long long)NX * NL;
        offF += (size_t)2 * NX * NL * NV;
        offC += (size_t)NX * NL;
        c->threads = std::max(c->threads, (NV + kWave - 1) / kWave * kWave);
    }
    c->cbase.push_back(cells);
    if (std::max(c->pop_base[0].back(), c->pop_base[1].back()) * 256 >= (1LL << 32)) {   // blocks of 256 threads
        delete c;
        return set_error(VLB_EINVAL, "batch too large for one population-kernel launch");
    }
    for (const auto& g : c->groups)   // one dispatch covers fewer than 2^32 work-items
        if (std::max(g.base.back(), g.bbase.back()) * kChanWaves * kWave >= (1LL << 32)) {
            delete c;
            return set_error(VLB_EINVAL, "batch too large for one stage launch (%lld blocks)", g.base.back());
        }
    c->state_n = offF;
    c->ncells = offC;
    size_t off = 0;
    for (int k = 0; k < 3; ++k) { c->off_F[k] = off; off = al256(off + c->state_n * sizeof(double)); }
    for (int k = 0; k < 3; ++k) {
        c->off_F32[k] = off;
        if (precision == VLB_MIXED) off = al256(off + c->state_n * sizeof(float));
    }
    c->off_desc32 = off; off = al256(off + (precision == VLB_MIXED ? B * sizeof(ChanDesc) : 0));
    c->off_sbase = off; off = al256(off + (B + 1) * sizeof(long long));
    c->off_rpart = off; off = al256(off + c->ncells * 4 * sizeof(double));
    c->off_resid = off; off = al256(off + B * sizeof(double));
    c->off_diag = off; off = al256(off + c->ncells * 5 * sizeof(double));
    c->off_fld = off; off = al256(off + c->fld_n * sizeof(double));
    c->off_tab = off; off = al256(off + c->tab.size() * sizeof(double));
    c->off_desc = off; off = al256(off + B * sizeof(ChanDesc));
    for (auto& g : c->groups) {
        g.off_ilist = off; off = al256(off + g.ilist.size() * sizeof(int));
        g.off_base = off; off = al256(off + g.base.size() * sizeof(long long));
        g.off_bbase = off; off = al256(off + g.bbase.size() * sizeof(long long));
    }
    c->off_cbase = off; off = al256(off + (B + 1) * sizeof(long long));
    for (int fm = 0; fm < 2; ++fm) {
        c->off_pop_ilist[fm] = off; off = al256(off + c->pop_ilist[fm].size() * sizeof(int));
        c->off_pop_base[fm] = off; off = al256(off + c->pop_base[fm].size() * sizeof(long long));
    }
    c->total = off;
    if (alloc) {
        void* p = nullptr;
        if (hipMalloc(&p, c->total) != hipSuccess) {
            delete c;
            return set_error(VLB_ENOMEM, "hipMalloc(%zu) failed", c->total);
        }
        c->ws = (char*)p;
        c->owns = true;
        vlb_status s = channel_device_setup(c);
        if (s != VLB_OK) {
            (void)hipFree(c->ws);
            delete c;
            return s;
        }
    }
    *out = c;
    return VLB_OK;
}

// Tables, descriptors and launch lists into the workspace, and the rest state n = 1,
// u = 0, T = T_w written on the device.  Synchronises.
vlb_status channel_device_setup(vlb_channel* c) {
    const int B = c->B;
    const int precision = c->precision;
    hipError_t e = hipMemcpyAsync(c->dtab(), c->tab.data(), c->tab.size() * sizeof(double), hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ddesc(), c->desc.data(), B * sizeof(ChanDesc), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && precision == VLB_MIXED)
        e = hipMemcpyAsync(c->ddesc32(), c->desc32.data(), B * sizeof(ChanDesc), hipMemcpyHostToDevice, c->stream);
    std::vector<long long> sbase(B + 1);
    for (int i = 0; i < B; ++i) sbase[i] = c->desc[i].offF;
    sbase[B] = (long long)c->state_n;
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->dsbase(), sbase.data(), (B + 1) * sizeof(long long), hipMemcpyHostToDevice, c->stream);
    for (auto& g : c->groups) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ws + g.off_ilist, g.ilist.data(), g.ilist.size() * sizeof(int),
                               hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ws + g.off_base, g.base.data(), g.base.size() * sizeof(long long),
                               hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ws + g.off_bbase, g.bbase.data(), g.bbase.size() * sizeof(long long),
                               hipMemcpyHostToDevice, c->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->dcbase(), c->cbase.data(), (B + 1) * sizeof(long long), hipMemcpyHostToDevice,
                           c->stream);
    for (int fm = 0; fm < 2; ++fm) {
        if (e == hipSuccess && !c->pop_ilist[fm].empty())
            e = hipMemcpyAsync(c->ws + c->off_pop_ilist[fm], c->pop_ilist[fm].data(),
                               c->pop_ilist[fm].size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && !c->pop_ilist[fm].empty())
            e = hipMemcpyAsync(c->ws + c->off_pop_base[fm], c->pop_base[fm].data(),
                               c->pop_base[fm].size() * sizeof(long long), hipMemcpyHostToDevice, c->stream);
    }
    // rest state n = 1, u = 0, T = T_w, written on the device
    if (e == hipSuccess)
        e = launch_channel_rest((long long)c->state_n, c->stream, c->ddesc(), c->dsbase(), B, c->dtab(), c->F(0));
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return set_error(VLB_EDEVICE, "channel set-up failed: %s", hipGetErrorString(e));
    return VLB_OK;
}
}  // namespace

vlb_status vlb_channel_destroy(vlb_channel* c) {
    if (!c) return VLB_OK;
    (void)hipStreamSynchronize(c->stream);
    for (hipGraphExec_t& g : c->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->ws && c->owns) (void)hipFree(c->ws);
    delete c;
    return VLB_OK;
}

vlb_status vlb_channel_set_graphs(vlb_channel* c, int enable) {
    if (!c) return set_error(VLB_EINVAL, "null channel batch");
    c->use_graphs = enable != 0;
    return VLB_OK;
}

vlb_status vlb_channel_info(const vlb_channel* c, int inst, int* N_lambda, int* N_xi, int* NV, double* dt,
                            size_t* state_offset) {
    if (!c || inst < 0 || inst >= c->B) return set_error(VLB_EINVAL, "bad instance");
    const ChanDesc& D = c->desc[inst];
    if (N_lambda) *N_lambda = D.NL;
    if (N_xi) *N_xi = D.NX;
    if (NV) *NV = D.NV;
    if (dt) *dt = D.dt;
    if (state_offset) *state_offset = (size_t)D.offF;
    return VLB_OK;
}

vlb_status vlb_channel_state_size(const vlb_channel* c, size_t* n) {
    if (!c || !n) return set_error(VLB_EINVAL, "null argument");
    *n = c->state_n;
    return VLB_OK;
}

vlb_status vlb_channel_set_state(vlb_channel* c, const double* host, size_t n) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || !host || n != c->state_n) return set_error(VLB_EINVAL, "state size mismatch");
    for (size_t x = 0; x < n; ++x)
        if (!std::isfinite(host[x])) return set_error(VLB_ENONFINITE, "non-finite value at element %zu", x);
    VLB_HIP_TRY(hipMemcpyAsync(c->F(0), host, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    c->have_resid = false;
    c->cur32 = false;
    c->polishing = false;
    return VLB_OK;
}

vlb_status vlb_channel_get_instance_state(vlb_channel* c, int inst, double* host, size_t n) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || inst < 0 || inst >= c->B || !host) return set_error(VLB_EINVAL, "bad instance");
    const ChanDesc& D = c->desc[inst];
    if (n != (size_t)2 * D.NX * D.NL * D.NV) return set_error(VLB_EINVAL, "instance state size mismatch");
    vlb_status s = channel_precision(c, false);
    if (s != VLB_OK) return s;
    VLB_HIP_TRY(hipMemcpyAsync(host, c->F(0) + D.offF, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    return VLB_OK;
}

vlb_status vlb_channel_set_instance_state(vlb_channel* c, int inst, const double* host, size_t n) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || inst < 0 || inst >= c->B || !host) return set_error(VLB_EINVAL, "bad instance");
    const ChanDesc& D = c->desc[inst];
    if (n != (size_t)2 * D.NX * D.NL * D.NV) return set_error(VLB_EINVAL, "instance state size mismatch");
    for (size_t x = 0; x < n; ++x)
        if (!std::isfinite(host[x])) return set_error(VLB_ENONFINITE, "non-finite value at element %zu", x);
    vlb_status s = channel_precision(c, false);
    if (s != VLB_OK) return s;
    VLB_HIP_TRY(hipMemcpyAsync(c->F(0) + D.offF, host, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    c->have_resid = false;
    c->polishing = false;
    return VLB_OK;
}

vlb_status vlb_channel_init_equilibrium(vlb_channel* c, int inst, const double* n, const double* u1,
                                        const double* u2, const double* T) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || inst < 0 || inst >= c->B || !n || !u1 || !u2 || !T) return set_error(VLB_EINVAL, "bad arguments");
    const ChanDesc& D = c->desc[inst];
    if (D.cartesian) return set_error(VLB_EINVAL, "instance %d is Cartesian-split", inst);
    const size_t nc = (size_t)D.NX * D.NL;
    std::vector<double> prof(4 * nc);
    const double* src[4] = {n, u1, u2, T};
    for (int q = 0; q < 4; ++q)
        for (size_t x = 0; x < nc; ++x) {
            const double v = src[q][x];
            if (!std::isfinite(v) || ((q == 0 || q == 3) && !(v > 0)))
                return set_error(VLB_EINVAL, "field %d at cell %zu: n and T must be positive and finite", q, x);
            prof[q * nc + x] = v;
        }
    vlb_status s = channel_precision(c, false);
    if (s != VLB_OK) return s;
    VLB_HIP_TRY(hipMemcpyAsync(c->fld(), prof.data(), prof.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    VLB_HIP_TRY(launch_channel_init_profile((long long)nc, c->stream, c->ddesc() + inst, c->dtab(), c->fld(), c->F(0)));
    VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    c->have_resid = false;
    c->polishing = false;
    return VLB_OK;
}

vlb_status vlb_channel_get_state(vlb_channel* c, double* host, size_t n) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || !host || n != c->state_n) return set_error(VLB_EINVAL, "state size mismatch");
    vlb_status s = channel_precision(c, false);
    if (s != VLB_OK) return s;
    VLB_HIP_TRY(hipMemcpyAsync(host, c->F(0), n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    return VLB_OK;
}

}  // extern "C"

namespace {

// One RK stage (or one application of L into the scratch buffer 1) on the current
// precision's buffers.
vlb_status channel_stage(vlb_channel* c, int stage, bool last, bool l_only) {
    const bool f32 = c->cur32;
    auto buf = [&](int k) -> void* { return f32 ? (void*)c->F32(k) : (void*)c->F(k); };
    ChanArgs A{};
    A.inst = f32 ? c->ddesc32() : c->ddesc();
    A.tab = c->dtab();
    A.rpart = nullptr;
    if (l_only) {
        A.Fin = buf(0); A.Fn = nullptr; A.Fout = buf(1);
        A.ca = 0; A.cb = 0; A.cc = 0; A.l_only = 1;
    } else if (stage == 0) {
        A.Fin = buf(0); A.Fn = nullptr; A.Fout = buf(1);
        A.ca = 0.0; A.cb = 1.0; A.cc = 1.0;
    } else if (stage == 1) {
        A.Fin = buf(1); A.Fn = buf(0); A.Fout = buf(2);
        A.ca = 0.75; A.cb = 0.25; A.cc = 0.25;
    } else {
        A.Fin = buf(2); A.Fn = buf(0); A.Fout = buf(0);
        A.ca = 1.0 / 3.0; A.cb = 2.0 / 3.0; A.cc = 2.0 / 3.0;
        if (last) A.rpart = c->rpart();
    }
    for (const auto& g : c->groups) {
        A.ilist = c->gilist(g);
        A.B = (int)g.ilist.size();
        A.base = c->gbase(g);
        VLB_HIP_TRY(launch_channel_stage(f32 ? 1 : 0, g.T1, g.T2, 0, g.base.back(), c->stream, A));
        A.base = c->gbbase(g);
        VLB_HIP_TRY(launch_channel_stage(f32 ? 1 : 0, g.T1, g.T2, 1, g.bbase.back(), c->stream, A));
    }
    for (int fm = 0; fm < 2; ++fm)   // population-kernel instances (FP64 only), per momentum form
        if (!c->pop_ilist[fm].empty()) {
            A.ilist = (const int*)(c->ws + c->off_pop_ilist[fm]);
            A.B = (int)c->pop_ilist[fm].size();
            A.base = (const long long*)(c->ws + c->off_pop_base[fm]);
            VLB_HIP_TRY(launch_pop_stage(fm, c->pop_base[fm].back(), c->stream, A));
        }
    return VLB_OK;
}

constexpr int kChanGraphSteps = 10;

// Capture kChanGraphSteps RK3 steps (every stage launch of the batch, no residual) of the
// current precision into an executable graph, on a private stream.
vlb_status channel_capture(vlb_channel* c, hipGraphExec_t* out) {
    if (!c->cap_stream) VLB_HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    vlb_status st = VLB_OK;
    if (e == hipSuccess) {
        for (int it = 0; it < kChanGraphSteps && st == VLB_OK; ++it)
            for (int stage = 0; stage < 3 && st == VLB_OK; ++stage) st = channel_stage(c, stage, false, false);
        e = hipStreamEndCapture(c->cap_stream, &g);
    }
    c->stream = user;
    if (st != VLB_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return set_error(VLB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return set_error(VLB_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    return VLB_OK;
}

vlb_status channel_steps(vlb_channel* c, long nsteps) {
    // all but the last step: replay captured chunks of kChanGraphSteps steps
    if (c->use_graphs && nsteps > kChanGraphSteps) {
        hipGraphExec_t& g = c->graph[c->cur32 ? 1 : 0];
        if (!g) {
            vlb_status s = channel_capture(c, &g);
            if (s != VLB_OK) return s;
        }
        while (nsteps > kChanGraphSteps) {
            VLB_HIP_TRY(hipGraphLaunch(g, c->stream));
            nsteps -= kChanGraphSteps;
        }
    }
    for (long it = 0; it < nsteps; ++it) {
        const bool last = it + 1 == nsteps;
        for (int st = 0; st < 3; ++st) {
            vlb_status s = channel_stage(c, st, last, false);
            if (s != VLB_OK) return s;
        }
        if (last) {
            VLB_HIP_TRY(launch_channel_reduce(c->B, c->stream, c->ddesc(), c->dtab(), c->rpart(), c->resid()));
            c->have_resid = true;
        }
    }
    return VLB_OK;
}

}  // namespace

extern "C" {

vlb_status vlb_channel_step(vlb_channel* c, long nsteps) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || nsteps < 0) return set_error(VLB_EINVAL, "bad arguments");
    vlb_status s = channel_precision(c, c->precision == VLB_MIXED);
    if (s != VLB_OK) return s;
    c->polishing = false;
    return channel_steps(c, nsteps);
}

vlb_status vlb_channel_step_fp64(vlb_channel* c, long nsteps) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || nsteps < 0) return set_error(VLB_EINVAL, "bad arguments");
    vlb_status s = channel_precision(c, false);
    if (s != VLB_OK) return s;
    return channel_steps(c, nsteps);
}

vlb_status vlb_channel_apply_L(vlb_channel* c, double* L, size_t n) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || !L || n != c->state_n) return set_error(VLB_EINVAL, "state size mismatch");
    vlb_status s = channel_stage(c, 0, false, true);
    if (s != VLB_OK) return s;
    if (c->cur32)   // L of the scaled populations times W_k is L of the populations
        VLB_HIP_TRY(launch_channel_convert(0, (long long)c->state_n, c->stream, c->ddesc32(), c->dsbase(), c->B,
                                           c->dtab(), c->F(1), c->F32(1)));
    VLB_HIP_TRY(hipMemcpyAsync(L, c->F(1), n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    return VLB_OK;
}

vlb_status vlb_channel_fp32_steps(const vlb_channel* c, long* n) {
    if (!c || !n) return set_error(VLB_EINVAL, "null argument");
    *n = c->fp32_steps;
    return VLB_OK;
}

vlb_status vlb_channel_residual(vlb_channel* c, double* r) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || !r) return set_error(VLB_EINVAL, "null argument");
    if (!c->have_resid) return set_error(VLB_ESTATE, "no step has recorded a residual yet");
    VLB_HIP_TRY(hipMemcpyAsync(r, c->resid(), c->B * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->B; ++i)
        if (!std::isfinite(r[i])) return set_error(VLB_ENONFINITE, "non-finite residual in instance %d", i);
    return VLB_OK;
}

vlb_status vlb_channel_moments(vlb_channel* c, int inst, double* n, double* u1, double* u2, double* T,
                               double* content) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || inst < 0 || inst >= c->B) return set_error(VLB_EINVAL, "bad instance");
    vlb_status s = channel_precision(c, false);
    if (s != VLB_OK) return s;
    VLB_HIP_TRY(launch_channel_diag(c->cbase.back(), c->threads, c->stream, c->ddesc(), c->dcbase(), c->B, c->dtab(),
                                    c->F(0), c->diag()));
    const ChanDesc& D = c->desc[inst];
    const size_t nc = (size_t)D.NX * D.NL;
    std::vector<double> h(nc * 5);
    VLB_HIP_TRY(hipMemcpyAsync(h.data(), c->diag() + (size_t)D.offC * 5, h.size() * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
    VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    double* outs[5] = {n, u1, u2, T, content};
    for (int q = 0; q < 5; ++q)
        if (outs[q])
            for (size_t x = 0; x < nc; ++x) outs[q][x] = h[x * 5 + q];
    return VLB_OK;
}

vlb_status vlb_channel_flow_fields(vlb_channel* c, int inst, double* ux, double* uy, double* P, double* psi,
                                   double* omega, double* Pw) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    if (!c || inst < 0 || inst >= c->B) return set_error(VLB_EINVAL, "bad instance");
    vlb_status s = channel_precision(c, false);
    if (s != VLB_OK) return s;
    VLB_HIP_TRY(launch_channel_diag(c->cbase.back(), c->threads, c->stream, c->ddesc(), c->dcbase(), c->B, c->dtab(),
                                    c->F(0), c->diag()));
    const ChanDesc& D = c->desc[inst];
    VLB_HIP_TRY(launch_channel_fields(D.NX, c->stream, c->ddesc() + inst, c->dtab(), c->diag(), c->fld()));
    const size_t nc = (size_t)D.NX * D.NL;
    const size_t len[6] = {nc, nc, nc, (size_t)D.NX * (D.NL + 1), nc, 2 * (size_t)D.NX};
    const size_t at[6] = {0, nc, 2 * nc, 4 * nc, 3 * nc, 4 * nc + (size_t)D.NX * (D.NL + 1)};
    double* outs[6] = {ux, uy, P, psi, omega, Pw};
    for (int q = 0; q < 6; ++q)
        if (outs[q])
            VLB_HIP_TRY(hipMemcpyAsync(outs[q], c->fld() + at[q], len[q] * sizeof(double), hipMemcpyDeviceToHost,
                                       c->stream));
    VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    return VLB_OK;
}

vlb_status vlb_channel_set_open_bc(vlb_channel* c, int inst, int end, double n, double T) {
    if (!c || inst < 0 || inst >= c->B || (end != 0 && end != 1) || !(n > 0) || !(T > 0) || !std::isfinite(n) ||
        !std::isfinite(T))
        return set_error(VLB_EINVAL, "bad arguments");
    vlb_channel_desc& d = c->d[inst];
    if (d.ends != 0) return set_error(VLB_EINVAL, "instance %d has flow-rate ends, not reservoirs", inst);
    AxisTables a1, a2;
    if (!build_axis(d.ax1.kind, d.ax1.Q, d.ax1.N, a1) || !build_axis(d.ax2.kind, d.ax2.Q, d.ax2.N, a2))
        return set_error(VLB_EINVAL, "axis construction failed");
    const int n1 = a1.nodes, n2 = a2.nodes, NV = n1 * n2;
    std::vector<double> g1(n1), g2(n2), f(2 * NV), fs(2 * NV);
    axis_equilibrium_host(a1, 0.0, T, g1.data());
    axis_equilibrium_host(a2, 0.0, T, g2.data());
    for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n2; ++b) {
            const int k = a * n2 + b;
            const double fw = g1[a] * g2[b];   // the same rounding as the tables built at creation
            f[k] = n * fw;
            f[NV + k] = n * (T * fw);
            const double iw = 1.0 / (a1.w[a] * a2.w[b]);
            fs[k] = f[k] * iw;
            fs[NV + k] = f[NV + k] * iw;
        }
    const ChanDesc& D = c->desc[inst];
    const size_t at = (size_t)D.offT + (end ? D.tfout : D.tfin);
    std::copy(f.begin(), f.end(), c->tab.begin() + at);
    if (c->ws)
        VLB_HIP_TRY(hipMemcpyAsync(c->dtab() + at, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice,
                                   c->stream));
    if (c->precision == VLB_MIXED) {
        const ChanDesc& E = c->desc32[inst];
        const size_t at32 = (size_t)E.offT + (end ? E.tfout : E.tfin);
        std::copy(fs.begin(), fs.end(), c->tab.begin() + at32);
        if (c->ws)
            VLB_HIP_TRY(hipMemcpyAsync(c->dtab() + at32, fs.data(), fs.size() * sizeof(double), hipMemcpyHostToDevice,
                                       c->stream));
    }
    if (c->ws) VLB_HIP_TRY(hipStreamSynchronize(c->stream));
    (end ? d.n_out : d.n_in) = n;
    c->have_resid = false;
    return VLB_OK;
}

vlb_status vlb_channel_total_mass(vlb_channel* c, double* Ntot) {
    if (!c || !Ntot) return set_error(VLB_EINVAL, "null argument");
    if (!c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    for (int i = 0; i < c->B; ++i) {
        const ChanDesc& D = c->desc[i];
        std::vector<double> content((size_t)D.NX * D.NL);
        vlb_status s = vlb_channel_moments(c, i, nullptr, nullptr, nullptr, nullptr, content.data());
        if (s != VLB_OK) return s;
        double acc = 0.0;
        for (double x : content) acc += x;
        Ntot[i] = acc;
    }
    return VLB_OK;
}

vlb_status vlb_channel_last_run_seconds(const vlb_channel* c, double* seconds) {
    if (!c || !seconds) return set_error(VLB_EINVAL, "null argument");
    *seconds = c->run_seconds;
    return VLB_OK;
}

namespace {
vlb_status channel_run(vlb_channel* c, double tol, long max_steps, int check_every, long* steps, double* r);
}

vlb_status vlb_channel_run_to_steady(vlb_channel* c, double tol, long max_steps, int check_every, long* steps,
                                     double* r) {
    if (c && !c->ws) return set_error(VLB_ESTATE, "no workspace bound");
    const auto t0 = std::chrono::steady_clock::now();
    const vlb_status s = channel_run(c, tol, max_steps, check_every, steps, r);
    if (c) c->run_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return s;
}

namespace {
vlb_status channel_run(vlb_channel* c, double tol, long max_steps, int check_every, long* steps, double* r) {
    if (!c || !(tol > 0) || max_steps < 1 || check_every < 1) return set_error(VLB_EINVAL, "bad arguments");
    std::vector<long> conv(c->B, -1);
    std::vector<double> res(c->B, INFINITY);
    long done = 0;
    vlb_status s = VLB_OK;
    if (c->precision == VLB_MIXED && !c->polishing) {
        // FP32 phase: stream the scaled FP32 state while the largest residual still falls;
        // stop at max(tol, 1e-5) or when it has not improved by 5% over three checks (the
        // FP32 rounding floor, about eps32 / dt), then continue in FP64
        s = channel_precision(c, true);
        if (s != VLB_OK) return s;
        double best = INFINITY;
        int stall = 0;
        while (done < max_steps) {
            const long n = std::min<long>(check_every, max_steps - done);
            s = channel_steps(c, n);
            if (s != VLB_OK) return s;
            done += n;
            s = vlb_channel_residual(c, res.data());
            if (s != VLB_OK) return s;
            const double worst = *std::max_element(res.begin(), res.end());
            if (worst < std::max(tol, 1e-5)) break;
            if (worst < 0.95 * best) {
                best = worst;
                stall = 0;
            } else if (++stall >= 3) {
                break;
            }
        }
        c->fp32_steps = done;
    }
    s = channel_precision(c, false);
    if (s != VLB_OK) return s;
    int remaining = c->B;
    while (done < max_steps && remaining > 0) {
        const long n = std::min<long>(check_every, max_steps - done);
        s = channel_steps(c, n);
        if (s != VLB_OK) return s;
        done += n;
        s = vlb_channel_residual(c, res.data());
        if (s != VLB_OK) return s;
        for (int i = 0; i < c->B; ++i)
            if (conv[i] < 0 && res[i] < tol) { conv[i] = done; --remaining; }
    }
    c->polishing = true;
    if (steps) std::copy(conv.begin(), conv.end(), steps);
    if (r) std::copy(res.begin(), res.end(), r);
    return remaining ? set_error(VLB_ENOTCONV, "%d channel(s) above tol after %ld steps", remaining, done) : VLB_OK;
}
}  // namespace

}  // extern "C"
