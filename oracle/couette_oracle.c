/*
 * Plain FP64 CPU oracle of the circular-Couette vielbein LB scheme (chi formulation, and
 * the f-tilde formulation of Sec. III for the comparison of Sec. V.C.2).
 * TEST INFRASTRUCTURE ONLY: nothing in the product library links or includes this
 * file, and this file includes nothing of the product library.
 *
 * What it computes, in the paper's order (arXiv:1708.05944):
 *   - Boltzmann-BGK equation in the chi form for cylindrical coordinates
 *     (Sec. V.A, Eq. boltz_couette_kom; stretched grids Eq. boltz_couette_str_kom),
 *     on reduced distributions f' and f'' (Sec. IV.A, Eqs. fred, macro_red);
 *   - moments n, u, T (Sec. IV.A) from quadrature sums (Eq. mom_quad);
 *   - polynomial equilibrium f'_eq = n g1 g2, f''_eq = T f'_eq (Sec. IV.D,
 *     Eqs. feq_red, eq_gak_H, eq_gak_hh);
 *   - diffuse-reflection walls (Sec. III.F, Eqs. weno_flux_eq, weno_populate,
 *     extrapol, nw);
 *   - epsilon-free WENO-5 fluxes (Sec. III.C, Eqs. weno5_flux, weno5_omega,
 *     weno_sigma and Table weno) and the flux difference of Eq. flux_kom_R /
 *     flux_kom_eta;
 *   - momentum-derivative force terms projected with the kernels of Sec. IV.C;
 *   - third-order TVD Runge-Kutta (Sec. III.A, Eq. rk3, Table rk3).
 * Readings where the paper is silent: WENO for V<0 is the
 * mirror image of the printed V>0 stencil; the 1/R factor of the force is the
 * cell value Gamma_s = 2/(R_{s+1/2}+R_{s-1/2}) (equal to 1/R_s on uniform grids);
 * f'' ghosts are T_w times the f' ghosts and wall-bound f'' uses the same
 * quadratic extrapolation; n_w uses f' only.
 *
 * Layout: F[d][s][k], d = 0 (f') / 1 (f''), s = 0..NR-1 (cell s+1 of the paper),
 * k = i*Q2 + j with i the axis-1 (radial) node and j the axis-2 (azimuthal) node.
 * Compiled with -O2 -ffp-contract=off and no fast-math.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int NR, Q1, Q2;          /* cells; nodes on axis 1 (p^R) and axis 2 (p^phi) */
    int kind1, kind2;        /* 0: full-range H, 1: half-range HH */
    int N1, N2;              /* equilibrium expansion orders */
    int Qh1, Qh2;            /* quadrature order Q of each axis (nodes = Q or 2Q) */
    const double *p1, *w1, *p2, *w2;
    const double *B1, *B2;   /* [nodes][N+1]: He_l(p) (H) or Phi^N_s(|p|) (HH) */
    const double *K1;        /* [Q1][Q1] d/dp^R kernel */
    const double *Kt2;       /* [Q2][Q2] d(p^phi .)/dp^phi kernel */
    const double *Rf;        /* [NR+1] face radii R_{s-1/2}, s = 1..NR+1 */
    const double *dchi;      /* [NR] (R_{s+1/2}^2 - R_{s-1/2}^2)/2 */
    const double *Gam;       /* [NR] inertial-force factor of each cell */
    double Kn;
    int tau_model;           /* 0: Kn sqrt(pi/8)/n, 1: Kn/(nT), 2: Kn/n */
    double u_in, T_in, u_out, T_out;   /* tangential wall speeds and temperatures */
    double weno_eps;         /* 0: the epsilon-free weights of Table weno; > 0: regularised */
    /* form 1: the f-tilde formulation (Sec. III, Eqs. boltz_cons and wf_def; Sec. V.A,
     * Eqs. boltz_couette_cons and boltz_couette_str_cons): the advective flux is
     * reconstructed from f-tilde = sqrt(g) f.  The state stays f; its time derivative is
     * the f-tilde equation's divided by sqrt(g) of the cell. */
    int form;
    const double *sqg;       /* [NR] sqrt(g) at the cell centres (R R'(eta); R on equal cells) */
    const double *ef;        /* [NR+1] e_eta^eta = 1 / R'(eta) at the faces (1 on equal cells) */
    double deta;             /* cell width in eta (delta R on equal cells) */
    double sqg_in, sqg_out;  /* sqrt(g) at the wall faces */
} couette_params;

/* ------------------------------------------------------------------ equilibrium */
/* P_s^+(x) = e^{-x^2} d^s/dx^s e^{x^2},  P_s^-(x) = e^{x^2} d^s/dx^s e^{-x^2}
 * (Sec. IV.D).  Built as coefficient arrays: if P_s = e^{-+x^2} D^s e^{+-x^2} then
 * P_{s+1} = P_s' +- 2x P_s. */
#define PMAX 24
static void p_poly(int sign, int smax, double c[PMAX][PMAX]) {
    memset(c, 0, sizeof(double) * PMAX * PMAX);
    c[0][0] = 1.0;
    for (int s = 0; s < smax; ++s) {
        for (int e = 0; e <= s; ++e) {
            if (e >= 1) c[s + 1][e - 1] += e * c[s][e];
            c[s + 1][e + 1] += sign * 2.0 * c[s][e];
        }
    }
}
static double poly_eval(const double* c, int deg, double x) {
    double r = 0.0;
    for (int e = deg; e >= 0; --e) r = r * x + c[e];
    return r;
}
static double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}
static double fact(int n) { double r = 1.0; for (int i = 2; i <= n; ++i) r *= i; return r; }

/* g_{a,k}(u, T) for one axis, Eq. eq_gak_H (kind 0) or Eq. eq_gak_hh (kind 1), m = 1. */
static void axis_eq(int kind, int Qh, int N, const double* p, const double* w,
                    const double* B, double u, double T, double* g) {
    int nodes = kind == 0 ? Qh : 2 * Qh;
    if (kind == 0) {
        for (int k = 0; k < nodes; ++k) {
            double acc = 0.0;
            for (int l = 0; l <= N; ++l) {
                double c = 0.0;
                for (int s = 0; s <= l / 2; ++s)
                    c += pow(T - 1.0, s) * pow(u, l - 2 * s) / (pow(2.0, s) * fact(s) * fact(l - 2 * s));
                acc += B[k * (N + 1) + l] * c;
            }
            g[k] = w[k] * acc;
        }
    } else {
        double Pp[PMAX][PMAX], Pm[PMAX][PMAX];
        p_poly(+1, N, Pp);
        p_poly(-1, N, Pm);
        for (int k = 0; k < nodes; ++k) {
            double zeta = (p[k] > 0 ? 1.0 : -1.0) * u / sqrt(2.0 * T);
            double acc = 0.0;
            for (int s = 0; s <= N; ++s) {
                double ps = poly_eval(Pp[s], s, zeta);
                double pstar = 0.0;
                for (int j = 0; j <= s - 1; ++j)
                    pstar += binom(s, j) * poly_eval(Pp[j], j, zeta) * poly_eval(Pm[s - j - 1], s - j - 1, zeta);
                double br = (1.0 + erf(zeta)) * ps + 2.0 / sqrt(M_PI) * exp(-zeta * zeta) * pstar;
                acc += pow(T / 2.0, 0.5 * s) * B[k * (N + 1) + s] * br;
            }
            g[k] = 0.5 * w[k] * acc;
        }
    }
}

/* f'_eq and f''_eq at one cell (Eq. feq_red and the line after it). */
void oracle_feq(const couette_params* P, double n, double u1, double u2, double T,
                double* fp, double* fpp) {
    double g1[256], g2[256];
    axis_eq(P->kind1, P->Qh1, P->N1, P->p1, P->w1, P->B1, u1, T, g1);
    axis_eq(P->kind2, P->Qh2, P->N2, P->p2, P->w2, P->B2, u2, T, g2);
    for (int i = 0; i < P->Q1; ++i)
        for (int j = 0; j < P->Q2; ++j) {
            double v = n * g1[i] * g2[j];
            fp[i * P->Q2 + j] = v;
            if (fpp) fpp[i * P->Q2 + j] = T * v;
        }
}

/* ------------------------------------------------------------------ moments */
/* n, u^1, u^2, T from Eqs. macro_red with m = 1: 3nT = sum(|xi|^2 f' + f''). */
void oracle_moments_cell(const couette_params* P, const double* fp, const double* fpp,
                         double* n, double* u1, double* u2, double* T) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int i = 0; i < P->Q1; ++i)
        for (int j = 0; j < P->Q2; ++j) {
            double f = fp[i * P->Q2 + j];
            s0 += f; s1 += P->p1[i] * f; s2 += P->p2[j] * f;
        }
    double uu1 = s1 / s0, uu2 = s2 / s0, e = 0;
    for (int i = 0; i < P->Q1; ++i)
        for (int j = 0; j < P->Q2; ++j) {
            double x1 = P->p1[i] - uu1, x2 = P->p2[j] - uu2;
            e += (x1 * x1 + x2 * x2) * fp[i * P->Q2 + j] + fpp[i * P->Q2 + j];
        }
    *n = s0; *u1 = uu1; *u2 = uu2; *T = e / (3.0 * s0);
}

static double tau_of(const couette_params* P, double n, double T) {
    if (P->tau_model == 0) return P->Kn * sqrt(M_PI / 8.0) / n;   /* Eq. tau_aoki */
    if (P->tau_model == 1) return P->Kn / (n * T);                /* Eq. hydro_tau */
    return P->Kn / n;                                             /* Sec. V.G benchmark */
}

/* ------------------------------------------------------------------ WENO-5 */
/* Flux at the face between c and d, upwinded from c: (a, b, c, d, e) are the five
 * cells of Eq. weno5_flux in upwind order (for V > 0 at face s+1/2:
 * F_{s-2}, F_{s-1}, F_s, F_{s+1}, F_{s+2}; for V < 0 the mirror image
 * F_{s+3}, F_{s+2}, F_{s+1}, F_s, F_{s-1}).  Weights of Eq. weno5_omega with the
 * epsilon-free limits of Table weno: if any smoothness indicator is exactly zero,
 * the ideal weights of the vanishing indicators are renormalised among themselves. */
void oracle_weno5_omega(double s1, double s2, double s3, double* w) {
    const double d1 = 0.1, d2 = 0.6, d3 = 0.3;   /* ideal weights */
    double w1, w2, w3;
    if (s1 == 0.0 || s2 == 0.0 || s3 == 0.0) {
        w1 = s1 == 0.0 ? d1 : 0.0;
        w2 = s2 == 0.0 ? d2 : 0.0;
        w3 = s3 == 0.0 ? d3 : 0.0;
    } else {
        w1 = d1 / (s1 * s1);
        w2 = d2 / (s2 * s2);
        w3 = d3 / (s3 * s3);
    }
    double sum = w1 + w2 + w3;
    w[0] = w1 / sum; w[1] = w2 / sum; w[2] = w3 / sum;
}

/* Smoothness indicators of Eq. weno_sigma for the upwind-ordered cells (a, b, c, d, e). */
void oracle_weno5_sigma(double a, double b, double c, double d, double e, double* s) {
    const double x1 = a - 2.0 * b + c, y1 = a - 4.0 * b + 3.0 * c;
    const double x2 = b - 2.0 * c + d, y2 = b - d;
    const double x3 = c - 2.0 * d + e, y3 = 3.0 * c - 4.0 * d + e;
    s[0] = 13.0 / 12.0 * (x1 * x1) + 0.25 * (y1 * y1);
    s[1] = 13.0 / 12.0 * (x2 * x2) + 0.25 * (y2 * y2);
    s[2] = 13.0 / 12.0 * (x3 * x3) + 0.25 * (y3 * y3);
}

/* WENO-5 face value with an optional regularisation (an extension; the paper's scheme
 * is eps = 0): when no indicator vanishes exactly, every indicator gets
 * eps (a^2 + b^2 + c^2 + d^2 + e^2) / 5 added before the weights are formed.  The added
 * term scales like the indicators, so the flux stays homogeneous of degree one in the
 * data; exactly vanishing indicators (e.g. the all-ghost wall stencil, which makes the
 * emitted flux exactly the ghost Maxwellian, Sec. III.F) keep the limits of Table weno.
 * eps -> infinity gives the ideal weights (0.1, 0.6, 0.3). */
double oracle_weno5_eps(double a, double b, double c, double d, double e, double eps) {
    double f1 = a / 3.0 - 7.0 / 6.0 * b + 11.0 / 6.0 * c;
    double f2 = -b / 6.0 + 5.0 / 6.0 * c + d / 3.0;
    double f3 = c / 3.0 + 5.0 / 6.0 * d - e / 6.0;
    double s[3];
    oracle_weno5_sigma(a, b, c, d, e, s);
    /* an indicator vanishes exactly when its three values are equal (Eq. weno_sigma is a
     * sum of squares of two independent differences); evaluating 3c - 4d + e in floating
     * point can leave a residue for equal values, which must not count as non-zero */
    if (a == b && b == c) s[0] = 0.0;
    if (b == c && c == d) s[1] = 0.0;
    if (c == d && d == e) s[2] = 0.0;
    if (eps > 0.0 && s[0] != 0.0 && s[1] != 0.0 && s[2] != 0.0) {
        const double add = eps * (a * a + b * b + c * c + d * d + e * e) / 5.0;
        s[0] += add;
        s[1] += add;
        s[2] += add;
    }
    double w[3];
    oracle_weno5_omega(s[0], s[1], s[2], w);
    return w[0] * f1 + w[1] * f2 + w[2] * f3;
}

double oracle_weno5(double a, double b, double c, double d, double e) { return oracle_weno5_eps(a, b, c, d, e, 0.0); }

/* ------------------------------------------------------------------ L[F] */
/* L[F] of Eq. L_def for the Couette chi formulation.  nw_res (may be NULL) gets the
 * inner and outer wall densities n_w of Eq. nw. */
void oracle_couette_L(const couette_params* P, const double* F, double* L, double* nw_res) {
    const int NR = P->NR, Q1 = P->Q1, Q2 = P->Q2, NV = Q1 * Q2;
    const size_t dsz = (size_t)NR * NV;
    /* extended arrays with 3 ghost cells on each side: E[d][s+3][k], s = -3..NR+2 */
    const int NE = NR + 6;
    double* E = (double*)calloc((size_t)2 * NE * NV, sizeof(double));
    double* feqw_in = (double*)calloc(NV, sizeof(double));
    double* feqw_out = (double*)calloc(NV, sizeof(double));
    double* mom = (double*)calloc((size_t)NR * 4, sizeof(double));
    double* fe = (double*)calloc((size_t)2 * NV, sizeof(double));
    const int ft = P->form == 1;
    for (int d = 0; d < 2; ++d)
        for (int s = 0; s < NR; ++s)
            for (int k = 0; k < NV; ++k) {
                const double f = F[d * dsz + (size_t)s * NV + k];
                /* f-tilde formulation: the reconstructed variable is sqrt(g) f */
                E[((size_t)d * NE + s + 3) * NV + k] = ft ? P->sqg[s] * f : f;
            }
#define EX(d, s, k) E[((size_t)(d) * NE + (s) + 3) * NV + (k)]

    /* 1. moments and relaxation time per cell */
    for (int s = 0; s < NR; ++s)
        oracle_moments_cell(P, F + (size_t)s * NV, F + dsz + (size_t)s * NV,
                            &mom[4 * s], &mom[4 * s + 1], &mom[4 * s + 2], &mom[4 * s + 3]);

    /* 2. walls (Sec. III.F).  Inner wall: face 1/2 (between ghost 0 and cell 1); the
     * emitted populations have p^R > 0.  Outer wall: face NR+1/2, emitted p^R < 0. */
    oracle_feq(P, 1.0, 0.0, P->u_in, P->T_in, feqw_in, NULL);
    oracle_feq(P, 1.0, 0.0, P->u_out, P->T_out, feqw_out, NULL);
    /* wall-bound populations: quadratic extrapolation, Eq. extrapol (both f' and f'') */
    for (int d = 0; d < 2; ++d)
        for (int k = 0; k < NV; ++k) {
            double F1 = EX(d, 0, k), F2 = EX(d, 1, k), F3 = EX(d, 2, k);
            EX(d, -1, k) = 3.0 * F1 - 3.0 * F2 + F3;
            EX(d, -2, k) = 6.0 * F1 - 8.0 * F2 + 3.0 * F3;
            EX(d, -3, k) = 0.0;
            double G1 = EX(d, NR - 1, k), G2 = EX(d, NR - 2, k), G3 = EX(d, NR - 3, k);
            EX(d, NR, k) = 3.0 * G1 - 3.0 * G2 + G3;
            EX(d, NR + 1, k) = 6.0 * G1 - 8.0 * G2 + 3.0 * G3;
            EX(d, NR + 2, k) = 0.0;
        }
    /* n_w from the zero-mass-flux condition, Eq. nw (the common factor R_wall cancels) */
    double num_in = 0, den_in = 0, num_out = 0, den_out = 0;
    for (int i = 0; i < Q1; ++i)
        for (int j = 0; j < Q2; ++j) {
            int k = i * Q2 + j;
            double pr = P->p1[i];
            if (pr > 0) {
                den_in += pr * feqw_in[k];
                /* outer wall, wall-bound (V > 0): flux at face NR+1/2 from cells NR-2..NR+2 */
                num_out += pr * oracle_weno5_eps(EX(0, NR - 3, k), EX(0, NR - 2, k), EX(0, NR - 1, k),
                                                 EX(0, NR, k), EX(0, NR + 1, k), P->weno_eps);
            } else if (pr < 0) {
                den_out += pr * feqw_out[k];
                /* inner wall, wall-bound (V < 0): mirrored stencil F_3, F_2, F_1, F_0, F_-1 */
                num_in += pr * oracle_weno5_eps(EX(0, 2, k), EX(0, 1, k), EX(0, 0, k), EX(0, -1, k), EX(0, -2, k), P->weno_eps);
            }
        }
    /* f-tilde: the emitted ghosts hold sqrt(g_wall) n_w f_eq, whose flux balances the
     * reconstructed wall-bound flux of f-tilde */
    const double gin = ft ? P->sqg_in : 1.0, gout = ft ? P->sqg_out : 1.0;
    double nw_in = -num_in / (gin * den_in), nw_out = -num_out / (gout * den_out);
    if (nw_res) { nw_res[0] = nw_in; nw_res[1] = nw_out; }
    /* emitted populations: ghost cells hold the wall Maxwellian, Eq. weno_populate */
    for (int i = 0; i < Q1; ++i)
        for (int j = 0; j < Q2; ++j) {
            int k = i * Q2 + j;
            double pr = P->p1[i];
            if (pr > 0)
                for (int g = -3; g <= -1; ++g) {
                    EX(0, g, k) = gin * (nw_in * feqw_in[k]);
                    EX(1, g, k) = gin * (P->T_in * nw_in * feqw_in[k]);
                }
            if (pr < 0)
                for (int g = NR; g <= NR + 2; ++g) {
                    EX(0, g, k) = gout * (nw_out * feqw_out[k]);
                    EX(1, g, k) = gout * (P->T_out * nw_out * feqw_out[k]);
                }
        }

    /* 3. per cell: advection (Eq. flux_kom_eta form), force, BGK */
    for (int d = 0; d < 2; ++d)
        for (int s = 0; s < NR; ++s) {
            double n = mom[4 * s], u1 = mom[4 * s + 1], u2 = mom[4 * s + 2], T = mom[4 * s + 3];
            double tau = tau_of(P, n, T);
            oracle_feq(P, n, u1, u2, T, fe, fe + NV);
            const double* Fc = F + d * dsz + (size_t)s * NV;
            for (int i = 0; i < Q1; ++i)
                for (int j = 0; j < Q2; ++j) {
                    int k = i * Q2 + j;
                    double pr = P->p1[i], pp = P->p2[j];
                    double fl, fr;   /* fluxes at faces s-1/2 and s+1/2 (paper cells s+1) */
                    if (pr > 0) {
                        fl = oracle_weno5_eps(EX(d, s - 3, k), EX(d, s - 2, k), EX(d, s - 1, k), EX(d, s, k), EX(d, s + 1, k), P->weno_eps);
                        fr = oracle_weno5_eps(EX(d, s - 2, k), EX(d, s - 1, k), EX(d, s, k), EX(d, s + 1, k), EX(d, s + 2, k), P->weno_eps);
                    } else {
                        fl = oracle_weno5_eps(EX(d, s + 2, k), EX(d, s + 1, k), EX(d, s, k), EX(d, s - 1, k), EX(d, s - 2, k), P->weno_eps);
                        fr = oracle_weno5_eps(EX(d, s + 3, k), EX(d, s + 2, k), EX(d, s + 1, k), EX(d, s, k), EX(d, s - 1, k), P->weno_eps);
                    }
                    /* chi form: Eq. flux_kom_R / flux_kom_eta; f-tilde form: Eq. flux_cons_R /
                     * flux_cons_eta, divided by sqrt(g) of the cell */
                    double adv = ft ? pr * (P->ef[s + 1] * fr - P->ef[s] * fl) / (P->deta * P->sqg[s])
                                    : pr * (P->Rf[s + 1] * fr - P->Rf[s] * fl) / P->dchi[s];
                    double kf = 0.0, ktf = 0.0;
                    for (int ip = 0; ip < Q1; ++ip) kf += P->K1[i * Q1 + ip] * Fc[ip * Q2 + j];
                    for (int jp = 0; jp < Q2; ++jp) ktf += P->Kt2[j * Q2 + jp] * Fc[i * Q2 + jp];
                    double force = P->Gam[s] * (pp * pp * kf - pr * ktf);
                    L[d * dsz + (size_t)s * NV + k] = -adv - force - (Fc[k] - fe[d * NV + k]) / tau;
                }
        }
#undef EX
    free(E); free(feqw_in); free(feqw_out); free(mom); free(fe);
}

/* ------------------------------------------------------------------ RK3 */
/* nsteps of the third-order TVD Runge-Kutta scheme of Eq. rk3 (Table rk3), in place. */
void oracle_couette_rk3(const couette_params* P, double* F, double dt, long nsteps) {
    const size_t n = (size_t)2 * P->NR * P->Q1 * P->Q2;
    double* L = (double*)malloc(n * sizeof(double));
    double* F1 = (double*)malloc(n * sizeof(double));
    double* F2 = (double*)malloc(n * sizeof(double));
    for (long it = 0; it < nsteps; ++it) {
        oracle_couette_L(P, F, L, NULL);
        for (size_t x = 0; x < n; ++x) F1[x] = F[x] + dt * L[x];
        oracle_couette_L(P, F1, L, NULL);
        for (size_t x = 0; x < n; ++x) F2[x] = 0.75 * F[x] + 0.25 * F1[x] + 0.25 * dt * L[x];
        oracle_couette_L(P, F2, L, NULL);
        for (size_t x = 0; x < n; ++x) F[x] = F[x] / 3.0 + 2.0 / 3.0 * F2[x] + 2.0 / 3.0 * dt * L[x];
    }
    free(L); free(F1); free(F2);
}
