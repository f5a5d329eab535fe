// Velocity-space tables of the mixed-quadrature LB models, built on the host in
// long double (x87 80-bit) when a velocity set is created.
//
// Construction route (independent of any other table generator):
//   * recurrence coefficients of the orthonormal polynomials for the weight
//     omega(x) = exp(-x^2/2)/sqrt(2 pi): exact for the full line (alpha = 0,
//     beta_l = l); for the half line [0, inf) by the discretised Stieltjes
//     procedure over a composite Gauss-Legendre rule on [0, 40];
//   * nodes = eigenvalues of the Jacobi matrix (Sturm-sequence bisection), i.e. the
//     roots of He_Q (Sec. IV.B) or of the half-range polynomial h_Q (Eq. hh_roots);
//   * weights = Christoffel numbers 1 / sum_{l<Q} phi_l(x)^2 of the orthonormal
//     family (equal to Eqs. w_H and w_hh);
//   * derivative kernels K (d/dp) and Kt (d(p .)/dp) from Sec. IV.C, Eqs. df_K_H,
//     df_K_hh, dfp_K_H, dfp_K_hh, written with the orthonormal recurrence values
//     (h_{l,0} = h_l(0), h_{l,l}/h_{l+1,l+1} = sqrt(beta_{l+1}), a_l = 1/sqrt(beta_{l+1}));
//   * equilibrium basis B[k][l] = w_k phi_l(|p_k|) and the monomial coefficients
//     needed to turn moments of the shifted Gaussian into expansion coefficients
//     (Sec. IV.D, Eqs. eq_gak_H, eq_gak_hh).
#include <cmath>
#include <cstring>
#include <vector>

#include "vlb_internal.h"

namespace vlb {

using ld = long double;

namespace {

const ld kPi = 3.141592653589793238462643383279502884L;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<ld>& x, std::vector<ld>& w) {
    x.assign(n, 0);
    w.assign(n, 0);
    auto legendre = [n](ld z, ld& pn, ld& dpn) {
        ld p0 = 1, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        pn = p1;
        dpn = n * (z * p1 - p0) / (z * z - 1);
    };
    for (int i = 0; i < n; ++i) {
        ld z = std::cos(kPi * (i + 0.75L) / (n + 0.5L)), pn, dpn;
        for (int it = 0; it < 60; ++it) {
            legendre(z, pn, dpn);
            const ld dz = pn / dpn;
            z -= dz;
            if (std::fabs(dz) <= 4e-19L) break;
        }
        legendre(z, pn, dpn);
        x[i] = z;
        w[i] = 2 / ((1 - z * z) * dpn * dpn);
    }
}

// Recurrence coefficients alpha[0..L-1], beta[0..L-1] (beta[0] = total mass) of the
// monic orthogonal polynomials for omega on [0, inf): discretised Stieltjes.
void half_line_recurrence(int L, std::vector<ld>& alpha, std::vector<ld>& beta) {
    std::vector<ld> gx, gw;
    gauss_legendre(24, gx, gw);
    const int panels = 160;
    const ld X = 40.0L, h = X / panels;
    std::vector<ld> x, w;
    for (int p = 0; p < panels; ++p)
        for (size_t i = 0; i < gx.size(); ++i) {
            ld xi = p * h + 0.5L * h * (gx[i] + 1);
            x.push_back(xi);
            w.push_back(0.5L * h * gw[i] * std::exp(-0.5L * xi * xi) / std::sqrt(2 * kPi));
        }
    const size_t M = x.size();
    std::vector<ld> pm(M, 0), pc(M, 1), pn(M);
    alpha.assign(L, 0);
    beta.assign(L, 0);
    ld norm_prev = 1;
    for (int k = 0; k < L; ++k) {
        ld nrm = 0, xn = 0;
        for (size_t m = 0; m < M; ++m) {
            nrm += w[m] * pc[m] * pc[m];
            xn += w[m] * x[m] * pc[m] * pc[m];
        }
        alpha[k] = xn / nrm;
        beta[k] = k == 0 ? nrm : nrm / norm_prev;
        norm_prev = nrm;
        for (size_t m = 0; m < M; ++m) {
            pn[m] = (x[m] - alpha[k]) * pc[m] - (k == 0 ? 0 : beta[k] * pm[m]);
            pm[m] = pc[m];
            pc[m] = pn[m];
        }
    }
}

// Eigenvalues of the symmetric tridiagonal matrix (diag a[0..n-1], off-diagonal b[1..n-1]),
// ascending, by Sturm-sequence bisection.
std::vector<ld> tridiag_eigs(const std::vector<ld>& a, const std::vector<ld>& b, int n) {
    ld lo = a[0], hi = a[0];
    for (int i = 0; i < n; ++i) {
        ld r = (i > 0 ? std::fabs(b[i]) : 0) + (i + 1 < n ? std::fabs(b[i + 1]) : 0);
        lo = std::fmin(lo, a[i] - r);
        hi = std::fmax(hi, a[i] + r);
    }
    auto count_below = [&](ld x) {
        int c = 0;
        ld d = 1;
        for (int i = 0; i < n; ++i) {
            d = a[i] - x - (i > 0 ? b[i] * b[i] / d : 0);
            if (d == 0) d = -1e-300L;
            if (d < 0) ++c;
        }
        return c;
    };
    std::vector<ld> ev(n);
    for (int k = 0; k < n; ++k) {
        ld l = lo, r = hi;
        for (int it = 0; it < 200; ++it) {
            ld m = 0.5L * (l + r);
            if (m == l || m == r) break;
            if (count_below(m) > k) r = m; else l = m;
        }
        ev[k] = 0.5L * (l + r);
    }
    return ev;
}

// Orthonormal values phi_0..phi_L at x from the recurrence (alpha, beta).
void ortho_values(const std::vector<ld>& alpha, const std::vector<ld>& beta, int L, ld x, ld* out) {
    out[0] = 1 / std::sqrt(beta[0]);
    if (L >= 1) out[1] = (x - alpha[0]) * out[0] / std::sqrt(beta[1]);
    for (int l = 1; l < L; ++l)
        out[l + 1] = ((x - alpha[l]) * out[l] - std::sqrt(beta[l]) * out[l - 1]) / std::sqrt(beta[l + 1]);
}

}  // namespace

// Builds all tables of one axis.  Returns false on invalid (kind, Q, N).
bool build_axis(int kind, int Q, int N, AxisTables& t) {
    if ((kind != 0 && kind != 1) || Q < 1 || Q > kMaxQ || N < 0 || N >= Q || N > kMaxN) return false;
    t.kind = kind;
    t.Q = Q;
    t.N = N;
    t.nodes = kind == 0 ? Q : 2 * Q;
    const int L = Q + 1;  // need phi_0..phi_Q
    std::vector<ld> alpha(L + 1), beta(L + 1);
    if (kind == 0) {
        for (int l = 0; l <= L; ++l) { alpha[l] = 0; beta[l] = l == 0 ? 1 : l; }
    } else {
        half_line_recurrence(L + 1, alpha, beta);
    }
    // nodes: eigenvalues of the Q x Q Jacobi matrix
    std::vector<ld> a(Q), b(Q, 0);
    for (int i = 0; i < Q; ++i) { a[i] = alpha[i]; if (i > 0) b[i] = std::sqrt(beta[i]); }
    std::vector<ld> x = tridiag_eigs(a, b, Q);
    std::vector<ld> p(t.nodes), w(t.nodes);
    std::vector<std::vector<ld>> phi(t.nodes, std::vector<ld>(L + 1));
    for (int i = 0; i < Q; ++i) {
        p[i] = x[i];
        if (kind == 1) p[Q + i] = -x[i];
    }
    for (int k = 0; k < t.nodes; ++k) {
        ld ax = kind == 1 ? std::fabs(p[k]) : p[k];
        ortho_values(alpha, beta, L, ax, phi[k].data());
        ld s = 0;
        for (int l = 0; l < Q; ++l) s += phi[k][l] * phi[k][l];
        w[k] = 1 / s;
    }
    t.p.assign(t.nodes, 0);
    t.w.assign(t.nodes, 0);
    for (int k = 0; k < t.nodes; ++k) { t.p[k] = (double)p[k]; t.w[k] = (double)w[k]; }

    // kernels
    const int n = t.nodes;
    t.K.assign((size_t)n * n, 0);
    t.Kt.assign((size_t)n * n, 0);
    if (kind == 0) {
        // He_l = sqrt(l!) phi_l; 1/l! He_{l+1}(x) He_l(y) = sqrt(l+1) phi_{l+1}(x) phi_l(y)
        for (int k = 0; k < n; ++k)
            for (int kp = 0; kp < n; ++kp) {
                ld acc = 0, acct = 0;
                for (int l = 0; l < Q; ++l) acc += std::sqrt((ld)(l + 1)) * phi[k][l + 1] * phi[kp][l];
                for (int l = 0; l + 1 < Q; ++l) {
                    // (1/l!) He_{l+1}(x)[He_{l+1}(y) + l He_{l-1}(y)]
                    ld term = (l + 1) * phi[k][l + 1] * phi[kp][l + 1];
                    if (l >= 1) term += std::sqrt((ld)(l + 1) * l) * phi[k][l + 1] * phi[kp][l - 1];
                    acct += term;
                }
                t.K[(size_t)k * n + kp] = (double)(-w[k] * acc);
                t.Kt[(size_t)k * n + kp] = (double)(-w[k] * acct);
            }
    } else {
        std::vector<ld> h0(L + 1);
        ortho_values(alpha, beta, L, 0.0L, h0.data());                      // h_{l,0} = h_l(0)
        std::vector<ld> ratio(L + 1), aa(L + 1);
        for (int l = 0; l < L; ++l) { ratio[l] = std::sqrt(beta[l + 1]); aa[l] = 1 / ratio[l]; }  // h_ll/h_{l+1,l+1}, a_l
        const ld s2pi = std::sqrt(2 * kPi);
        std::vector<ld> phi0(n, 0);                                          // Phi^Q_0(|p_k|)
        for (int k = 0; k < n; ++k)
            for (int l = 0; l <= Q; ++l) phi0[k] += h0[l] * phi[k][l];
        for (int k = 0; k < n; ++k) {
            const int sk = k < Q ? 1 : -1;
            for (int kp = 0; kp < n; ++kp) {
                const int skp = kp < Q ? 1 : -1;
                const bool same = sk == skp;
                ld acc = 0;
                if (same)
                    for (int l = 0; l + 1 < Q; ++l) {
                        ld tail = 0;
                        for (int s = l + 1; s < Q; ++s) tail += h0[s] * phi[k][s];
                        acc += phi[kp][l] * (h0[l] / s2pi * tail - ratio[l] * phi[k][l + 1]);
                    }
                acc -= phi0[k] * phi0[kp] / (2 * s2pi);
                t.K[(size_t)k * n + kp] = (double)(w[k] * sk * acc);
                ld acct = 0;
                if (same)
                    for (int l = 0; l < Q; ++l) {
                        ld term = l * phi[kp][l];
                        if (l >= 1) term += (h0[l] * h0[l] + h0[l - 1] * h0[l - 1]) / (aa[l - 1] * s2pi) * phi[kp][l - 1];
                        if (l >= 2) term += phi[kp][l - 2] / (aa[l - 1] * aa[l - 2]);
                        acct += phi[k][l] * term;
                    }
                t.Kt[(size_t)k * n + kp] = (double)(-w[k] * acct);
            }
        }
    }

    // equilibrium basis: B[k][l] = w_k phi_l(|p_k|) (l = 0..N) and, per axis kind, the
    // map from Gaussian moments to expansion coefficients:
    //   full range: coefficient of phi_l is E[phi_l(X)] = E[He_l]/sqrt(l!)  (recurrence on device)
    //   half range: coefficient of phi_l is sum_s c[l][s] M_s, c[l][s] = monomial coefficient
    //               of x^s in phi_l, M_s = int_0^inf x^s g(x) dx (M_s by recurrence on device)
    t.B.assign((size_t)n * (N + 1), 0);
    for (int k = 0; k < n; ++k)
        for (int l = 0; l <= N; ++l) t.B[(size_t)k * (N + 1) + l] = (double)(w[k] * phi[k][l]);
    t.C.assign((size_t)(N + 1) * (N + 1), 0);
    {
        // monomial coefficients of phi_l from the recurrence
        std::vector<std::vector<ld>> c(N + 2, std::vector<ld>(N + 2, 0));
        c[0][0] = 1 / std::sqrt(beta[0]);
        if (N >= 1) { c[1][1] = c[0][0] / std::sqrt(beta[1]); c[1][0] = -alpha[0] * c[0][0] / std::sqrt(beta[1]); }
        for (int l = 1; l < N; ++l)
            for (int s = 0; s <= l + 1; ++s) {
                ld v = (s >= 1 ? c[l][s - 1] : 0) - alpha[l] * c[l][s] - std::sqrt(beta[l]) * c[l - 1][s];
                c[l + 1][s] = v / std::sqrt(beta[l + 1]);
            }
        for (int l = 0; l <= N; ++l)
            for (int s = 0; s <= l; ++s) t.C[(size_t)l * (N + 1) + s] = (double)c[l][s];
    }
    // inverse square roots of l! for the full-range coefficient normalisation
    t.invsqrtfact.assign(N + 1, 0);
    {
        ld f = 1;
        for (int l = 0; l <= N; ++l) { if (l > 0) f *= l; t.invsqrtfact[l] = (double)(1 / std::sqrt(f)); }
    }
    return true;
}

// Host evaluation of the axis equilibrium g_k(u, T) (used for wall tables and the
// host-side initial states): same expansion the device uses.
void axis_equilibrium_host(const AxisTables& t, double u, double T, double* g) {
    const int N = t.N;
    ld coef_p[kMaxN + 1], coef_m[kMaxN + 1];
    if (t.kind == 0) {
        // a_l = E[He_l(X)]/l!, X ~ N(u, T):  l a_l = u a_{l-1} + (T-1) a_{l-2}
        ld a[kMaxN + 2];
        a[0] = 1;
        if (N >= 1) a[1] = u;
        for (int l = 2; l <= N; ++l) a[l] = (u * a[l - 1] + (T - 1.0L) * a[l - 2]) / l;
        // coefficient of phi_l = He_l/sqrt(l!) is E[He_l]/sqrt(l!) = a_l sqrt(l!)
        for (int l = 0; l <= N; ++l) coef_p[l] = coef_m[l] = a[l] / t.invsqrtfact[l];
    } else {
        for (int sgn = 0; sgn < 2; ++sgn) {
            ld uu = sgn == 0 ? u : -u;
            // M_s = int_0^inf x^s g(x) dx, g = N(uu, T):
            //   M_0 = (1 + erf(uu/sqrt(2T)))/2,  M_1 = uu M_0 + T g(0),
            //   M_s = uu M_{s-1} + (s-1) T M_{s-2}
            ld M[kMaxN + 2];
            ld g0 = std::exp(-uu * uu / (2 * T)) / std::sqrt(2 * kPi * T);
            M[0] = 0.5L * (1 + std::erf((double)(uu / std::sqrt(2 * T))));
            if (N >= 1) M[1] = uu * M[0] + T * g0;
            for (int s = 2; s <= N; ++s) M[s] = uu * M[s - 1] + (s - 1) * T * M[s - 2];
            ld* co = sgn == 0 ? coef_p : coef_m;
            for (int l = 0; l <= N; ++l) {
                ld acc = 0;
                for (int s = 0; s <= l; ++s) acc += t.C[(size_t)l * (N + 1) + s] * M[s];
                co[l] = acc;
            }
        }
    }
    for (int k = 0; k < t.nodes; ++k) {
        const ld* co = (t.kind == 1 && k >= t.Q) ? coef_m : coef_p;
        ld acc = 0;
        for (int l = 0; l <= N; ++l) acc += t.B[(size_t)k * (N + 1) + l] * co[l];
        g[k] = (double)acc;
    }
}

}  // namespace vlb
