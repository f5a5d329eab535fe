/* Plain FP64 oracle of the expanding-channel hot path (TEST INFRASTRUCTURE ONLY).
 *
 * Busuioc & Ambrus, arXiv:1708.05944, Sec. VI: the reduced Boltzmann-BGK equation in
 * the coordinates lambda = x / (1 + phi(xi)), xi = y with the orthonormal triad of
 * Sec. VI.A (Eqs. canalie_phat, canalie_boltz, canalie_V, chi_canalie), written in
 * conservative form
 *   d_t f + d_lambda (V^lambda f) + d_chi (V^xi f)
 *        - G_lxx [ (p^xi)^2 d f/d p^lambda - p^lambda d(f p^xi)/d p^xi ]
 *        - G_xll [ (p^lambda)^2 d f/d p^xi - p^xi d(f p^lambda)/d p^lambda ] = -(f - f_eq)/tau,
 * with G_xll = -G_lxl (antisymmetry of the connection), G_lxl and G_lxx discretised as
 * in Sec. VI.A so that a uniform Maxwellian is an exact solution, tau = Kn/(nT)
 * (Eq. canalie_tau), epsilon-free WENO-5 fluxes (Sec. III.C) upwinded by the sign of the
 * face velocity, diffuse walls at lambda = -1 and +1 (Sec. VI.C.4 applied at both walls:
 * the full channel width), and reservoir ends: at the inlet (outlet) the populations
 * entering the domain see ghost cells at f_eq(n_in (n_out), 0, T_w) and the leaving
 * ones a zeroth-order extrapolation (the construction of Sec. VI.C.1 with the
 * density fixed instead of the flow rate).
 *
 * The paper's own boundary conditions are options: the upper half of the channel,
 * lambda in [0, 1], with specular reflection at the centreline (Sec. VI.C.3: ghost cells
 * -1, -2, -3 hold cells 0, 1, 2 with p^lambda reversed), and flow-rate ends (Sec. VI.C.1,
 * VI.C.2): per lambda row s the entering populations see f_eq(n_s, u_s, T_w) with the
 * Cartesian velocity (u^x, u^y) = (0, Q(lambda_s)) of the parabolic profile Q(lambda) =
 * 3 Q0 / (H (1 + phi)) (1 - 4 lambda^2 / H^2), H = 2 (Eqs. canalie_inlet, canalie_outlet),
 * the leaving ones a zeroth-order extrapolation, and n_s makes the row's flow rate
 * sum_k p^y F_face equal Q(lambda_s) (p^y = V^xi / (1 + phi) at the face).
 *
 * State layout: F[d][p][s][k], d = f' / f'', p = xi cell (0..NX-1), s = lambda cell
 * (0..NL-1), k = i*Q2 + j (i: p^lambda node, j: p^xi node).  Compiled together with
 * couette_oracle.c (velocity-set machinery shared within the oracle). */
#include "couette_oracle.c"

typedef struct {
    couette_params vs;        /* velocity set, Kn, tau model, weno_eps (NR, faces unused) */
    int NL, NX;               /* cells across (lambda) and along (xi) the channel */
    const double *Kt1;        /* [Q1][Q1] d(p^lambda .)/d p^lambda kernel */
    const double *K2;         /* [Q2][Q2] d/d p^xi kernel */
    const double *lam_f;      /* [NL+1] lambda faces */
    const double *phi_c, *dphi_c;   /* [NX] phi and phi' at the xi cell centres */
    const double *phi_f, *dphi_f;   /* [NX+1] at the xi faces */
    const double *dchi;       /* [NX] chi(xi_{p+1/2}) - chi(xi_{p-1/2}), d chi = (1 + phi) d xi */
    double n_in, n_out, T_w;  /* reservoir densities, wall / reservoir temperature */
    int half;                 /* 1: lambda in [0, 1], specular centreline at lambda = 0 */
    int ends;                 /* 0: reservoirs at n_in / n_out; 1: flow-rate profile of Q0 */
    double Q0;                /* flow rate through half of the cross-section (ends = 1) */
} channel_params;

/* V^xi at xi-face f of lambda cell s for the velocity (pl, px), Eq. canalie_V */
static double v_xi(const channel_params* P, int s, int f, double pl, double px) {
    const double lam = 0.5 * (P->lam_f[s] + P->lam_f[s + 1]);
    const double a = lam * P->dphi_f[f];
    return (1.0 + P->phi_f[f]) * (px - a * pl) / sqrt(1.0 + a * a);
}

/* Cartesian flow velocity (0, Q) in the triad at an xi face: with a = lambda phi' and
 * c = 1 / sqrt(1 + a^2), p^x = c (p^lambda + a p^xi), p^y = c (p^xi - a p^lambda), so
 * u^lambda = -a c Q and u^xi = c Q. */
static void end_velocity(const channel_params* P, int s, int f, double Q, double* ul, double* ux) {
    const double lam = 0.5 * (P->lam_f[s] + P->lam_f[s + 1]);
    const double a = lam * P->dphi_f[f], c = 1.0 / sqrt(1.0 + a * a);
    *ul = -a * c * Q;
    *ux = c * Q;
}

/* prescribed flow rate of row s at the end face f (0 or NX), H = 2 */
static double end_flow_rate(const channel_params* P, int s, int f) {
    const double lam = 0.5 * (P->lam_f[s] + P->lam_f[s + 1]), H = 2.0;
    return 3.0 * P->Q0 / (H * (1.0 + P->phi_f[f])) * (1.0 - 4.0 * lam * lam / (H * H));
}

/* L[F] (Eq. canalie_boltz for f' and f''); xi_flux (may be NULL) gets, for every xi
 * face f = 0..NX, sum_s dlambda_s sum_k V^xi F_face of f' (particle flux through the
 * cross-section); nw (may be NULL) the wall densities [NX][2] (lower, upper; 0 for the
 * specular centreline); row_flow (may be NULL) the flow rate sum_k p^y F_face of every
 * lambda row at the inlet and outlet faces [2][NL]. */
void oracle_channel_L2(const channel_params* P, const double* F, double* L, double* xi_flux, double* nw,
                       double* row_flow) {
    const couette_params* V = &P->vs;
    const int NL = P->NL, NX = P->NX, Q1 = V->Q1, Q2 = V->Q2, NV = Q1 * Q2;
    const int EL = NL + 6, EX = NX + 6;
    const size_t dsz = (size_t)NX * NL * NV;
    /* extended array with 3 ghost cells around: G[d][p+3][s+3][k] (corners unused) */
    double* G = (double*)calloc((size_t)2 * EX * EL * NV, sizeof(double));
    double* mom = (double*)calloc((size_t)NX * NL * 4, sizeof(double));
    double* fe = (double*)calloc((size_t)2 * NV, sizeof(double));
    double* feq_w = (double*)calloc((size_t)2 * NV, sizeof(double));
    double* feq_in = (double*)calloc((size_t)2 * NV, sizeof(double));
    double* feq_out = (double*)calloc((size_t)2 * NV, sizeof(double));
#define GX(d, p, s, k) G[((((size_t)(d) * EX + (p) + 3) * EL + (s) + 3) * NV) + (k)]
#define FX(d, p, s, k) F[(size_t)(d) * dsz + ((size_t)(p) * NL + (s)) * NV + (k)]
    for (int d = 0; d < 2; ++d)
        for (int p = 0; p < NX; ++p)
            for (int s = 0; s < NL; ++s)
                for (int k = 0; k < NV; ++k) GX(d, p, s, k) = FX(d, p, s, k);

    /* 1. moments per cell */
    for (int p = 0; p < NX; ++p)
        for (int s = 0; s < NL; ++s) {
            double* m = mom + ((size_t)p * NL + s) * 4;
            oracle_moments_cell(V, &FX(0, p, s, 0), &FX(1, p, s, 0), &m[0], &m[1], &m[2], &m[3]);
        }

    /* 2a. walls at lambda = -1 (face s = -1/2, emitted p^lambda > 0) and lambda = +1
     * (face NL - 1/2, emitted p^lambda < 0), per xi column: wall-bound ghosts by the
     * quadratic extrapolation (Eq. extrapol), n_w by zero mass flux (Eq. nw; the factor
     * sqrt(1 + lambda_w^2 phi'^2) / (1 + phi) of V^lambda is common and cancels) */
    oracle_feq(V, 1.0, 0.0, 0.0, P->T_w, feq_w, feq_w + NV);
    oracle_feq(V, P->n_in, 0.0, 0.0, P->T_w, feq_in, feq_in + NV);
    oracle_feq(V, P->n_out, 0.0, 0.0, P->T_w, feq_out, feq_out + NV);
    for (int p = 0; p < NX; ++p) {
        for (int d = 0; d < 2; ++d)
            for (int k = 0; k < NV; ++k) {
                const double F1 = GX(d, p, 0, k), F2 = GX(d, p, 1, k), F3 = GX(d, p, 2, k);
                GX(d, p, -1, k) = 3.0 * F1 - 3.0 * F2 + F3;
                GX(d, p, -2, k) = 6.0 * F1 - 8.0 * F2 + 3.0 * F3;
                GX(d, p, -3, k) = 0.0;
                const double H1 = GX(d, p, NL - 1, k), H2 = GX(d, p, NL - 2, k), H3 = GX(d, p, NL - 3, k);
                GX(d, p, NL, k) = 3.0 * H1 - 3.0 * H2 + H3;
                GX(d, p, NL + 1, k) = 6.0 * H1 - 8.0 * H2 + 3.0 * H3;
                GX(d, p, NL + 2, k) = 0.0;
            }
        double num_lo = 0, den_lo = 0, num_hi = 0, den_hi = 0;
        for (int i = 0; i < Q1; ++i)
            for (int j = 0; j < Q2; ++j) {
                const int k = i * Q2 + j;
                const double pl = V->p1[i];
                if (pl > 0) {
                    den_lo += pl * feq_w[k];
                    num_hi += pl * oracle_weno5_eps(GX(0, p, NL - 3, k), GX(0, p, NL - 2, k), GX(0, p, NL - 1, k),
                                                    GX(0, p, NL, k), GX(0, p, NL + 1, k), V->weno_eps);
                } else if (pl < 0) {
                    den_hi += pl * feq_w[k];
                    num_lo += pl * oracle_weno5_eps(GX(0, p, 2, k), GX(0, p, 1, k), GX(0, p, 0, k), GX(0, p, -1, k),
                                                    GX(0, p, -2, k), V->weno_eps);
                }
            }
        const double nw_lo = P->half ? 0.0 : -num_lo / den_lo, nw_hi = -num_hi / den_hi;
        if (nw) { nw[2 * p] = nw_lo; nw[2 * p + 1] = nw_hi; }
        for (int i = 0; i < Q1; ++i)
            for (int j = 0; j < Q2; ++j) {
                const int k = i * Q2 + j;
                const double pl = V->p1[i];
                for (int g = 1; g <= 3; ++g) {
                    if (P->half) {
                        /* specular centreline: cell g - 1 with p^lambda reversed */
                        const int kbar = ((i + V->Qh1) % Q1) * Q2 + j;
                        GX(0, p, -g, k) = GX(0, p, g - 1, kbar);
                        GX(1, p, -g, k) = GX(1, p, g - 1, kbar);
                    } else if (pl > 0) {
                        GX(0, p, -g, k) = nw_lo * feq_w[k];
                        GX(1, p, -g, k) = nw_lo * feq_w[NV + k];
                    }
                    if (pl < 0) {
                        GX(0, p, NL - 1 + g, k) = nw_hi * feq_w[k];
                        GX(1, p, NL - 1 + g, k) = nw_hi * feq_w[NV + k];
                    }
                }
            }
    }
    /* 2b. reservoir ends, per lambda row: entering populations (V^xi > 0 at the inlet
     * face, < 0 at the outlet face) see the reservoir Maxwellian, leaving ones the
     * nearest interior cell */
    for (int s = 0; s < NL; ++s) {
        if (P->ends == 1) {
            /* flow-rate ends: the Maxwellians of the row's profile velocity at unit density,
             * scaled by the density that makes the row's flow rate the prescribed one */
            double ul, ux;
            end_velocity(P, s, 0, end_flow_rate(P, s, 0), &ul, &ux);
            oracle_feq(V, 1.0, ul, ux, P->T_w, feq_in, feq_in + NV);
            end_velocity(P, s, NX, end_flow_rate(P, s, NX), &ul, &ux);
            oracle_feq(V, 1.0, ul, ux, P->T_w, feq_out, feq_out + NV);
            double lin = 0, din = 0, lout = 0, dout = 0;
            for (int i = 0; i < Q1; ++i)
                for (int j = 0; j < Q2; ++j) {
                    const int k = i * Q2 + j;
                    const double pyi = v_xi(P, s, 0, V->p1[i], V->p2[j]) / (1.0 + P->phi_f[0]);
                    const double pyo = v_xi(P, s, NX, V->p1[i], V->p2[j]) / (1.0 + P->phi_f[NX]);
                    if (pyi > 0) din += feq_in[k] * pyi;
                    else lin += GX(0, 0, s, k) * pyi;
                    if (pyo < 0) dout += feq_out[k] * pyo;
                    else lout += GX(0, NX - 1, s, k) * pyo;
                }
            const double nin = (end_flow_rate(P, s, 0) - lin) / din;
            const double nout = (end_flow_rate(P, s, NX) - lout) / dout;
            for (int k = 0; k < 2 * NV; ++k) {
                feq_in[k] *= nin;
                feq_out[k] *= nout;
            }
        }
        for (int i = 0; i < Q1; ++i)
            for (int j = 0; j < Q2; ++j) {
                const int k = i * Q2 + j;
                const double vin = v_xi(P, s, 0, V->p1[i], V->p2[j]);
                const double vout = v_xi(P, s, NX, V->p1[i], V->p2[j]);
                for (int d = 0; d < 2; ++d)
                    for (int g = 1; g <= 3; ++g) {
                        GX(d, -g, s, k) = vin > 0 ? feq_in[d * NV + k] : GX(d, 0, s, k);
                        GX(d, NX - 1 + g, s, k) = vout < 0 ? feq_out[d * NV + k] : GX(d, NX - 1, s, k);
                    }
            }
    }
    if (row_flow)
        for (int x = 0; x < 2 * NL; ++x) row_flow[x] = 0.0;

    /* face values of the xi-fluxes of f' for the cross-section fluxes */
    if (xi_flux)
        for (int f = 0; f <= NX; ++f) xi_flux[f] = 0.0;

    /* 3. per cell: advection, force, BGK */
    for (int d = 0; d < 2; ++d)
        for (int p = 0; p < NX; ++p)
            for (int s = 0; s < NL; ++s) {
                const double* m = mom + ((size_t)p * NL + s) * 4;
                const double n = m[0], T = m[3];
                const double tau = tau_of(V, n, T);
                oracle_feq(V, n, m[1], m[2], T, fe, fe + NV);
                const double lam = 0.5 * (P->lam_f[s] + P->lam_f[s + 1]);
                const double dlam = P->lam_f[s + 1] - P->lam_f[s];
                const double ph = P->phi_c[p], dph = P->dphi_c[p];
                /* metric factors of V^lambda at the lambda faces (xi at the cell centre) */
                const double al = sqrt(1.0 + P->lam_f[s] * P->lam_f[s] * dph * dph) / (1.0 + ph);
                const double ar = sqrt(1.0 + P->lam_f[s + 1] * P->lam_f[s + 1] * dph * dph) / (1.0 + ph);
                /* connection coefficients (Sec. VI.A, discrete form) */
                const double bl = lam * P->dphi_f[p], br = lam * P->dphi_f[p + 1];
                const double ql = (1.0 + P->phi_f[p]) / sqrt(1.0 + bl * bl);
                const double qr = (1.0 + P->phi_f[p + 1]) / sqrt(1.0 + br * br);
                const double G_lxl = (qr - ql) / P->dchi[p];
                const double G_lxx = -(sqrt(1.0 + P->lam_f[s + 1] * P->lam_f[s + 1] * dph * dph) -
                                       sqrt(1.0 + P->lam_f[s] * P->lam_f[s] * dph * dph)) / (dlam * (1.0 + ph)) +
                                     lam / P->dchi[p] * (P->dphi_f[p + 1] * qr - P->dphi_f[p] * ql);
                const double G_xll = -G_lxl;
                const double* Fc = &FX(d, p, s, 0);
                for (int i = 0; i < Q1; ++i)
                    for (int j = 0; j < Q2; ++j) {
                        const int k = i * Q2 + j;
                        const double pl = V->p1[i], px = V->p2[j];
                        /* lambda faces, upwinded by the sign of p^lambda */
                        double Fl, Fr;
                        if (pl > 0) {
                            Fl = oracle_weno5_eps(GX(d, p, s - 3, k), GX(d, p, s - 2, k), GX(d, p, s - 1, k),
                                                  GX(d, p, s, k), GX(d, p, s + 1, k), V->weno_eps);
                            Fr = oracle_weno5_eps(GX(d, p, s - 2, k), GX(d, p, s - 1, k), GX(d, p, s, k),
                                                  GX(d, p, s + 1, k), GX(d, p, s + 2, k), V->weno_eps);
                        } else {
                            Fl = oracle_weno5_eps(GX(d, p, s + 2, k), GX(d, p, s + 1, k), GX(d, p, s, k),
                                                  GX(d, p, s - 1, k), GX(d, p, s - 2, k), V->weno_eps);
                            Fr = oracle_weno5_eps(GX(d, p, s + 3, k), GX(d, p, s + 2, k), GX(d, p, s + 1, k),
                                                  GX(d, p, s, k), GX(d, p, s - 1, k), V->weno_eps);
                        }
                        const double adv_l = pl * (ar * Fr - al * Fl) / dlam;
                        /* xi faces, upwinded by the sign of V^xi at each face */
                        double Vx[2], Fx[2];
                        for (int e = 0; e < 2; ++e) {
                            const int f = p + e;            /* face index: p - 1/2 -> p, p + 1/2 -> p + 1 */
                            Vx[e] = v_xi(P, s, f, pl, px);
                            if (Vx[e] > 0)
                                Fx[e] = oracle_weno5_eps(GX(d, f - 3, s, k), GX(d, f - 2, s, k), GX(d, f - 1, s, k),
                                                         GX(d, f, s, k), GX(d, f + 1, s, k), V->weno_eps);
                            else
                                Fx[e] = oracle_weno5_eps(GX(d, f + 2, s, k), GX(d, f + 1, s, k), GX(d, f, s, k),
                                                         GX(d, f - 1, s, k), GX(d, f - 2, s, k), V->weno_eps);
                        }
                        const double adv_x = (Vx[1] * Fx[1] - Vx[0] * Fx[0]) / P->dchi[p];
                        if (row_flow && d == 0) {
                            if (p == 0) row_flow[s] += Vx[0] * Fx[0] / (1.0 + P->phi_f[0]);
                            if (p == NX - 1) row_flow[NL + s] += Vx[1] * Fx[1] / (1.0 + P->phi_f[NX]);
                        }
                        if (xi_flux && d == 0) {
                            xi_flux[p + 1] += dlam * Vx[1] * Fx[1] / (p + 1 < NX ? 2.0 : 1.0);
                            xi_flux[p] += dlam * Vx[0] * Fx[0] / (p > 0 ? 2.0 : 1.0);
                        }
                        /* momentum derivatives by the projection kernels (Sec. IV.C) */
                        double k1 = 0, kt1 = 0, k2 = 0, kt2 = 0;
                        for (int ip = 0; ip < Q1; ++ip) {
                            k1 += V->K1[i * Q1 + ip] * Fc[ip * Q2 + j];
                            kt1 += P->Kt1[i * Q1 + ip] * Fc[ip * Q2 + j];
                        }
                        for (int jp = 0; jp < Q2; ++jp) {
                            k2 += P->K2[j * Q2 + jp] * Fc[i * Q2 + jp];
                            kt2 += V->Kt2[j * Q2 + jp] * Fc[i * Q2 + jp];
                        }
                        const double force = G_lxx * (px * px * k1 - pl * kt2) + G_xll * (pl * pl * k2 - px * kt1);
                        L[(size_t)d * dsz + ((size_t)p * NL + s) * NV + k] =
                            -adv_l - adv_x + force - (Fc[k] - fe[d * NV + k]) / tau;
                    }
            }
#undef GX
#undef FX
    free(G); free(mom); free(fe); free(feq_w); free(feq_in); free(feq_out);
}

void oracle_channel_L(const channel_params* P, const double* F, double* L, double* xi_flux, double* nw) {
    oracle_channel_L2(P, F, L, xi_flux, nw, NULL);
}

/* nsteps SSP-RK3 steps (Eq. rk3) in place */
void oracle_channel_rk3(const channel_params* P, double* F, double dt, long nsteps) {
    const size_t n = (size_t)2 * P->NX * P->NL * P->vs.Q1 * P->vs.Q2;
    double* F1 = (double*)malloc(n * sizeof(double));
    double* F2 = (double*)malloc(n * sizeof(double));
    double* L = (double*)malloc(n * sizeof(double));
    for (long it = 0; it < nsteps; ++it) {
        oracle_channel_L(P, F, L, NULL, NULL);
        for (size_t x = 0; x < n; ++x) F1[x] = F[x] + dt * L[x];
        oracle_channel_L(P, F1, L, NULL, NULL);
        for (size_t x = 0; x < n; ++x) F2[x] = 0.75 * F[x] + 0.25 * F1[x] + 0.25 * dt * L[x];
        oracle_channel_L(P, F2, L, NULL, NULL);
        for (size_t x = 0; x < n; ++x) F[x] = F[x] / 3.0 + 2.0 / 3.0 * F2[x] + 2.0 / 3.0 * dt * L[x];
    }
    free(F1); free(F2); free(L);
}
