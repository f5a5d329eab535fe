/*
 * vlb.h -- C ABI of the MI355X vielbein lattice-Boltzmann library (libvlb.so).
 *
 * The library advances the finite-difference lattice Boltzmann model of
 * Busuioc & Ambrus, arXiv:1708.05944: the Boltzmann-BGK equation in the conservative
 * vielbein ("chi") form (Sec. II.B, Eq. boltz_noncons; Sec. III, Eq. numsch_eq),
 * written for circular Couette flow (Sec. V.A, Eq. boltz_couette_kom and, on
 * stretched grids, Eq. boltz_couette_str_kom), on the reduced distributions f' and
 * f'' (Sec. IV.A, Eq. fred) over mixed half-/full-range Gauss-Hermite velocity sets
 * HH(N;Q) x H(N;Q) (Sec. IV.B, Eq. model).  One time step is the third-order TVD
 * Runge-Kutta scheme (Sec. III.A, Eq. rk3); each stage evaluates moments, the
 * polynomial equilibrium (Sec. IV.D), diffuse-reflection walls (Sec. III.F),
 * epsilon-free WENO-5 fluxes (Sec. III.C) and the projected inertial force
 * (Sec. IV.C) on the GPU.
 *
 * Conventions
 *   - Units: m = k_B = T_w(reference) = 1; momenta in units of sqrt(m k_B T_0).
 *   - A "batch" holds B independent Couette instances of possibly different grid
 *     sizes and velocity sets; a single solver is a batch of one.
 *   - State layout (host and device): instances one after the other; instance b is
 *     a block [2][N_R][NV] of doubles: f' then f'', cell s = 0..N_R-1 (cell s+1 of
 *     the paper, cell-centred, Sec. V.C.1), velocity k = i*Q2 + j with i the node of
 *     axis 1 (radial momentum p^R) and j the node of axis 2 (azimuthal p^phi).  Node
 *     order per axis: full range -> ascending roots of He_Q; half range -> the Q
 *     positive roots ascending, then their mirror images (Sec. IV.B).  Stored values
 *     are the weighted populations f_ij = w_i w_j f(p_i, p_j)/(omega(p_i) omega(p_j)).
 *   - Errors: every call returns a vlb_status; no C++ exception crosses the ABI.
 *     vlb_last_error() gives a thread-local message for the last failure.
 *   - Ownership: the caller owns every host array it passes; the library never keeps
 *     a host pointer past the call.  Device memory is allocated by the library on
 *     creation, or supplied by the caller with vlb_batch_bind_workspace (e.g. a
 *     torch tensor), in which case the caller keeps it alive until destroy.
 *   - Streams: work is enqueued on the hipStream_t given at creation (NULL = the
 *     default stream).  Calls that return host data synchronise that stream.
 *   - Handles are not thread-safe; use one handle per thread.
 */
#ifndef VLB_H
#define VLB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VLB_OK = 0,
    VLB_EINVAL = -1,       /* invalid argument (sizes, orders, pointers, unknown enum) */
    VLB_ENOMEM = -2,       /* host or device allocation failed / workspace too small */
    VLB_EDEVICE = -3,      /* a HIP runtime call or kernel launch failed */
    VLB_ESTATE = -4,       /* call not valid in the handle's current state */
    VLB_ENOTCONV = -5,     /* run_to_steady stopped at max_steps above tolerance */
    VLB_ENONFINITE = -6,   /* NaN or Inf found in the state or residual */
    VLB_EUNSTABLE = -7     /* requested dt violates the stability limits */
} vlb_status;

/* One momentum axis: kind 0 = full-range Gauss-Hermite H(N;Q), kind 1 = half-range
 * HH(N;Q) (2Q nodes); N is the expansion order of the equilibrium, 0 <= N < Q
 * (Sec. IV.D, Eq. norder_limit), N <= 4; 1 <= Q <= 64. */
typedef struct {
    int kind;
    int Q;
    int N;
} vlb_axis;

/* Relaxation-time models tau(n, T) of the BGK term (Eq. BGK). */
enum {
    VLB_TAU_AOKI = 0,      /* tau = Kn sqrt(pi/8) / n   (Sec. V.F, Eq. tau_aoki) */
    VLB_TAU_HYDRO = 1,     /* tau = Kn / (n T)          (Sec. V.D, Eq. hydro_tau) */
    VLB_TAU_KN = 2         /* tau = Kn / n              (Sec. V.G benchmark runs) */
};

/* Precision of a batch.  VLB_FP64: every stage in FP64.  VLB_MIXED: the batch also
 * holds an FP32 copy of the state, stored as the populations divided by their
 * quadrature weight w_i w_j (O(1) values); its stage kernels stream and compute in FP32
 * while moment sums, the wall mass balance (Eq. nw) and the residual accumulate in
 * FP64.  Results handed to the caller (state, moments, L) are always FP64. */
enum { VLB_FP64 = 0, VLB_MIXED = 1 };

/* One circular-Couette instance (Sec. V).  Grid: N_R >= 3 cells between R_in < R_out;
 * A = 0 gives an equidistant grid, 0 < A < 1 the tanh stretching of Sec. III.B
 * (Eqs. eta_def, eta_inout) with centre parameter delta in [0, 1].  ax1 is the radial
 * axis, ax2 the azimuthal one; ax1.kind = 1 (half range) is the choice that resolves
 * the wall discontinuity (Sec. IV.B).  dt = 0 picks dt = cfl * min_s dchi_s /
 * (R_{s+1/2} max|p^R|).  Walls: tangential speeds u_in / u_out and temperatures
 * T_in / T_out of the inner and outer cylinder (Sec. III.F, Eq. diffuse_f).
 * weno_eps: 0 (the paper's epsilon-free WENO weights of Table weno), or > 0 for
 * regularised weights (an extension): when no smoothness indicator of a stencil
 * vanishes exactly, each gets weno_eps * (a^2 + b^2 + c^2 + d^2 + e^2) / 5 added (a..e
 * the stencil values), which removes the chatter of the epsilon-free weights that
 * stalls the residual near some steady states; stencils with a vanishing indicator
 * (the all-ghost wall stencil) keep the Table weno limits, so the wall mass balance
 * stays exact. */
typedef struct {
    double R_in, R_out;
    int N_R;
    double A, delta;
    vlb_axis ax1, ax2;
    double Kn;
    int tau_model;
    double dt, cfl;
    double u_in, T_in, u_out, T_out;
    double weno_eps;
    int form;     /* 0: the chi formulation (Sec. V.A, Eq. boltz_couette_kom), the method; 1: the
                   * f-tilde formulation (Sec. III, Eq. boltz_cons; Sec. V.A, Eqs. boltz_couette_cons,
                   * boltz_couette_str_cons), kept for the comparison of Sec. V.C.2: the advective
                   * flux is reconstructed from sqrt(g) f, sqrt(g) = R R'(eta) at cell centres,
                   * e_eta = 1/R'(eta) at faces, the emitted wall ghosts holding sqrt(g_wall) n_w
                   * f_eq; the state is f in both forms.  FP64 only; runs on the four-launch stage. */
} vlb_couette_desc;

typedef struct vlb_batch vlb_batch;

/* Creates B >= 1 instances; builds velocity sets and grids on the host, uploads
 * tables, allocates device memory unless defer_alloc != 0 (then bind a workspace
 * before any other call), and sets every instance to the rest state n = 1, u = 0,
 * T = T_in (Sec. V, initial state).  precision is VLB_FP64 or VLB_MIXED.  hip_stream is a
 * hipStream_t (may be NULL).  Errors: VLB_EINVAL for invalid descriptors (N_R < 3,
 * R_out <= R_in, invalid axes, Kn <= 0, dt < 0), VLB_EUNSTABLE if an explicit dt
 * exceeds the CFL limit of the instance, VLB_ENOMEM, VLB_EDEVICE. */
vlb_status vlb_batch_create_couette(vlb_batch** out, int B, const vlb_couette_desc* descs, int precision,
                                    void* hip_stream, int defer_alloc);
void vlb_batch_destroy(vlb_batch* b);

/* Bytes of device memory the batch needs, and binding of a caller-owned buffer of at
 * least that size (256-byte aligned).  Binding replaces library-owned memory and
 * resets the state to rest. */
vlb_status vlb_batch_workspace_bytes(const vlb_batch* b, size_t* bytes);
vlb_status vlb_batch_bind_workspace(vlb_batch* b, void* dev_ptr, size_t bytes);

/* Per-instance sizes: cells, velocities (NV = nodes1 * nodes2), axis node counts,
 * the time step in use, and the element offset of the instance in the state. */
vlb_status vlb_batch_info(const vlb_batch* b, int inst, int* N_R, int* NV, int* nodes1, int* nodes2, double* dt,
                          size_t* state_offset);
/* Total number of doubles of the state (sum over instances of 2 N_R NV). */
vlb_status vlb_batch_state_size(const vlb_batch* b, size_t* n_doubles);

/* Velocity set of one instance: nodes and weights of axis 1 / 2 (host arrays of
 * length nodes1 / nodes2). */
vlb_status vlb_batch_velocities(const vlb_batch* b, int inst, double* p1, double* w1, double* p2, double* w2);

/* Replace the wall parameters of one instance (side 0 = inner, 1 = outer). */
vlb_status vlb_set_wall(vlb_batch* b, int inst, int side, double u_tangential, double T_w);

/* Initialise instance inst (or all instances when inst = -1, arrays concatenated over
 * instances) to the local equilibrium f' = f'_eq(n, u, T), f'' = T f'_eq per cell
 * (Sec. IV.D).  Host arrays of N_R (or total cells) entries. */
vlb_status vlb_init_equilibrium(vlb_batch* b, int inst, const double* n, const double* u1, const double* u2,
                                const double* T);

/* Copy the whole state to / from a host array of vlb_batch_state_size doubles.
 * set_state rejects non-finite values with VLB_ENONFINITE. */
vlb_status vlb_set_state(vlb_batch* b, const double* host, size_t n);
vlb_status vlb_get_state(vlb_batch* b, double* host, size_t n);

/* Advance every instance by nsteps >= 0 RK3 steps, each with its own dt, in the batch's
 * streaming precision (FP32 for VLB_MIXED batches, converting the state on first use).
 * The last step records the steady-state residual r of each instance (see
 * vlb_residual).  Enqueued on the stream; returns without synchronising.
 * vlb_step_fp64 always steps in FP64 (converting a MIXED batch's state back first). */
vlb_status vlb_step(vlb_batch* b, long nsteps);
vlb_status vlb_step_fp64(vlb_batch* b, long nsteps);

/* One application of the operator L[F] of Eq. L_def (advection + force + BGK with the
 * diffuse walls) to the current state, in the precision the state currently lives in;
 * result written to the host array L (unscaled, same layout and size as the state).
 * The state is not modified.  Synchronises. */
vlb_status vlb_apply_L(vlb_batch* b, double* L, size_t n);

/* Macroscopic fields of one instance (host arrays of N_R; any may be NULL):
 * n, u^R, u^phi, T, T^{R phi}, q^R, q^phi (Sec. IV.A, Eq. macro_red).  Synchronises. */
vlb_status vlb_moments(vlb_batch* b, int inst, double* n, double* u1, double* u2, double* T, double* T12,
                       double* q1, double* q2);

/* Steady-state residual of the last recorded step of each instance (host array of B):
 * r = ||F^{n+1} - F^n||_W / (dt ||F^n||_W), ||F||_W^2 = sum_s dchi_s sum_k
 * (f'^2 + f''^2)/(w_i w_j).  VLB_ESTATE if no step was taken since the last state
 * change; VLB_ENONFINITE if any r is not finite.  Synchronises. */
vlb_status vlb_residual(vlb_batch* b, double* r);

/* Particle number per unit height and radian, N_tot = sum_s dchi_s n_s
 * (Sec. II.B, Eq. Ntot_def), per instance (host array of B).  Synchronises. */
vlb_status vlb_total_mass(vlb_batch* b, double* Ntot);

/* Step every instance until its residual is below tol, checking every check_every
 * steps, at most max_steps steps.  An instance whose residual is below tol at a check
 * retires: the stage kernels stop advancing it while the others run (on shorter cell runs
 * than vlb_batch_set_tile / vlb_batch_autotune chose once those left no longer fill the
 * 256 CUs; the chosen length is restored on return), so its state,
 * moments and residual stay those of the step at which it converged.  steps / r (host
 * arrays of B, may be NULL) receive that step count (or -1) and the last residual.  Returns
 * VLB_ENOTCONV if some instance did not converge.  The residual judged is always the
 * FP64 one of the plain solver (one FP64 RK3 step of the current iterate).
 * VLB_MIXED batches reach the FP64 steady state by defect correction: each check takes
 * one FP64 step (the residual), then the FP64 defect R = L[F] (Eq. L_def, one FP64
 * operator application) drives check_every - 1 FP32 steps of the correction equation
 * d delta/dt = R + J delta from delta = 0, J being the operator linearised about F
 * (advection, force and walls as for a state, BGK linearised about the FP64 moments),
 * with delta stored and streamed in FP32 at its own scale; then F += delta in FP64.  The
 * fixed point is the FP64 one (R = 0), so the final state is an FP64 steady state while
 * nearly every step streams FP32; vlb_mixed_fp32_steps reports the FP32 steps taken since
 * the state was last replaced.  Consecutive calls continue the same iteration.
 * Instances started from the surrogate (vlb_batch_warm_start) are watched: one whose
 * residual has set no new low (by 1 %) for the stall window (vlb_batch_set_stall_window,
 * default 10000 steps) is restarted from the cold rest state and continues as a cold
 * start (vlb_batch_warm_report). */
vlb_status vlb_run_to_steady(vlb_batch* b, double tol, long max_steps, int check_every, long* steps, double* r);
/* Wall-clock seconds of the last vlb_run_to_steady call on b (host clock around the whole
 * call, which synchronises at every check, so the device work is inside it); 0 before any. */
vlb_status vlb_batch_last_run_seconds(const vlb_batch* b, double* seconds);
vlb_status vlb_mixed_fp32_steps(const vlb_batch* b, long* n);
/* State of the defect correction per instance (host arrays of B, any may be NULL, not
 * all): the relaxation factor theta of its next update F += theta * delta (1: the full
 * correction; halved to at least 1/8 after three checks in a row without a new residual
 * low by 1 %, doubled back after eight in a row with one); the step of the current run at
 * which it left the correction for FP64 steps for good (-1: it has not); the FP32
 * correction steps it took in the current run.  An instance is put on a trial of FP64
 * steps (5 checks) when its update was just halved, or when its residual fell by less than
 * a factor 10 over the last 10 checks, at least 20 checks after its last trial (40, 80, ...
 * after each lost one); it keeps FP64 steps if its residual fell by a factor 2 over the
 * trial and decayed 1.5 times faster than under the correction over the checks before
 * (fp64_from is then the trial's first step), else it returns to the correction.  On FP64
 * steps, an instance that sets no new low for 20000 steps (plain stepping can settle
 * into a cycle that the relaxed correction damps) returns to the correction with theta =
 * 1/8.  1 / -1 / 0 for an FP64 batch or before a run. */
vlb_status vlb_mixed_report(const vlb_batch* b, double* theta, long* fp64_from, long* fp32_steps);

/* Host-side velocity-set tables of one axis, for checking against independent
 * implementations: nodes p, weights w (nodes entries), d/dp kernel K and d(p .)/dp
 * kernel Kt (nodes x nodes, row-major; Sec. IV.C).  nodes = Q (kind 0) or 2Q. */
vlb_status vlb_axis_tables(vlb_axis ax, double* p, double* w, double* K, double* Kt);

/* Cells per run of the stage kernel (1..32; default 16): each block sweeps runs of this
 * many consecutive cells, one thread per velocity.  Short runs give small instances more
 * parallel blocks; long runs amortise the 3-cell halo at each run end.
 * vlb_batch_autotune times `steps` steps three times for each cells-per-run value from 1 to
 * 32 on the batch itself (the state is saved to a device copy and restored), keeps the value
 * with the fastest of all these timings, and returns it with that time per step in ms.
 * Allocates a temporary device copy of the state. */
vlb_status vlb_batch_set_tile(vlb_batch* b, int cells_per_run);
vlb_status vlb_batch_get_tile(const vlb_batch* b, int* cells_per_run);
vlb_status vlb_batch_autotune(vlb_batch* b, int steps, int* chosen, double* ms_per_step);

/* Step graphs.  By default vlb_step replays a HIP graph of 10 captured RK3 steps
 * (captured once per precision on a private non-blocking stream at first use, then
 * launched on the batch's stream) for all but the last step of a call, which runs as
 * plain launches and records the residual.  enable = 0 makes every step plain
 * launches (bitwise the same results). */
vlb_status vlb_batch_set_graphs(vlb_batch* b, int enable);

/* Multi-step launches (off by default; max_blocks = 64 is the intended setting).  While
 * the stage kernel's block
 * list of the instances being stepped has at most max_blocks blocks (small batches, the
 * last instances of a run_to_steady) and the device can hold them all resident, a call
 * of two or more steps runs them in cooperative launches of up to 2000 whole RK3 steps
 * each, with a grid-wide barrier between stages, instead of three launches (or graph
 * nodes) per step: a small instance is bound by launch latency otherwise.  Results are
 * bitwise those of plain launches (the same per-block stage code).  Not used for
 * instances with large velocity sets, for the defect correction while it splits its
 * instances between FP64 and linearised FP32 steps, or while per-launch timing is on.
 * max_blocks = 0 turns it off.  Measured on the single-instance workload (64 cells, 32
 * velocities) it is no faster than graph replay: a step there is bound by the stage
 * kernel's own latency (about 16 us per stage, in the per-cell equilibrium set-up and the
 * cell sweep), not by launches. */
vlb_status vlb_batch_set_persistent(vlb_batch* b, int max_blocks);

/* Kernel timing for roofline reports.  When enabled, every launch of the stage kernel
 * is bracketed by HIP events recorded on the batch's stream; launches are grouped by
 * kernel instantiation.  vlb_timing_query synchronises the stream and returns, for up
 * to max_groups groups: the element width in bits of the instantiation (64 for the FP64
 * kernel, 32 for the FP32 kernel), the number of launches recorded, their summed duration in ms, and the algorithmic HBM
 * bytes they moved (each launch: per population of the instances it covers, one read
 * of the stage input, one read of F_n in stages 2 and 3, one write).  Querying clears
 * the record.  ngroups receives the number of groups with launches. */
vlb_status vlb_timing_enable(vlb_batch* b, int enable);
vlb_status vlb_timing_query(vlb_batch* b, int max_groups, int* ngroups, int* bits, long* launches, double* total_ms,
                            double* alg_bytes);

/* ---- Learned warm start (an addition to the method: the paper has no surrogate) ----
 *
 * A multilayer perceptron maps, per cell, the inputs
 *   (log10 Kn, u_w, beta = R_in/R_out, rho = (R - R_in)/(R_out - R_in)),
 * each mapped affinely from the box [-2, 1] x [0.05, 0.5] x [0.3, 0.8] x [0, 1] to
 * [-1, 1], to the steady fields ((n - 1) 10, u^R 10, u^phi / u_w, (T - 1) 10) at the
 * cell centre R.  Network: 4 inputs -> depth hidden layers of width units with SiLU
 * activations, silu(z) = z / (1 + e^-z) -> 4 linear outputs.  Parameters are FP32, in
 * the same order on host and device: for each layer, W[fan_in][fan_out] row-major, then
 * b[fan_out].  Training minimises the mean squared error over all outputs of a
 * mini-batch with Adam (b1 = 0.9, b2 = 0.999, eps = 1e-8, bias-corrected; Kingma & Ba
 * 2015) using FP32 matrix-core products; inference uses bfloat16 operands with FP32
 * accumulation.  The network works on its stream (created with), one call at a time.
 * The surrogate's family: inner wall moving tangentially (u_in > 0), outer wall at rest,
 * both walls at T_w = 1, VLB_TAU_AOKI. */
typedef struct vlb_mlp vlb_mlp;

/* Parameter count of a width x depth network (width 1..1024, depth 1..8). */
vlb_status vlb_mlp_param_count(int width, int depth, size_t* n);
/* Network with the given initial parameters (host array, param_count floats; the
 * caller draws them).  Allocates its parameters, Adam moments and gradient on the
 * device; activation buffers grow with the largest batch seen. */
vlb_status vlb_mlp_create(vlb_mlp** out, int width, int depth, const float* params, void* hip_stream);
vlb_status vlb_mlp_destroy(vlb_mlp* m);
vlb_status vlb_mlp_get_params(vlb_mlp* m, float* host, size_t n);
/* Replaces the parameters and clears the Adam state (moments and step count). */
vlb_status vlb_mlp_set_params(vlb_mlp* m, const float* host, size_t n);
/* Y[n][4] = network(X[n][4]), device arrays; bf16 = 1 rounds every layer's operands
 * (inputs and weights) to bfloat16 (nearest, ties to even), 0 computes in FP32. */
vlb_status vlb_mlp_forward(vlb_mlp* m, const float* X, long n, float* Y, int bf16);
/* Mean squared error of the network on device rows X[n][4] against T[n][4] and its
 * gradient (FP32 forward and reverse passes).  loss (host scalar) and grad (host,
 * param_count floats) may be NULL; the gradient also stays on the device for
 * vlb_mlp_adam_step.  Synchronises. */
vlb_status vlb_mlp_loss_grad(vlb_mlp* m, const float* X, const float* T, long n, float* loss, float* grad);
/* One Adam step with learning rate lr on the given host gradient (param_count floats,
 * e.g. one summed over several devices), or on the last device gradient if grad is NULL. */
vlb_status vlb_mlp_adam_step(vlb_mlp* m, const float* grad, float lr);
/* Adam steps over mini-batches: rows order[0..norder) of the device samples X, T
 * (nsamples rows each) taken batch rows at a time (the last mini-batch may be
 * shorter); every order entry must be in [0, nsamples).  mean_loss (may be NULL)
 * receives the mean of the mini-batch losses.  Synchronises. */
vlb_status vlb_mlp_train(vlb_mlp* m, const float* X, const float* T, long nsamples, const int* order, long norder,
                         int batch, float lr, float* mean_loss);
/* Training samples from the batch's current state (normally a steady state): the
 * inputs and targets above for every cell of every instance, host arrays X[ncells][4],
 * T[ncells][4] with ncells the batch's total cell count.  Every instance must be in
 * the surrogate's family (VLB_EINVAL otherwise).  Synchronises. */
vlb_status vlb_batch_surrogate_samples(vlb_batch* b, float* X, float* T, size_t ncells);
/* Replaces every instance's state by an initial state: for an instance in the
 * surrogate's family, the local equilibrium of the network's fields (bfloat16
 * inference) with n rescaled so that sum_s dchi_s n_s equals the cold start's (the
 * steady state of the closed cell depends on this conserved particle number, Eq.
 * Ntot_def) and u^R = 0; for the others, and for any instance the acceptance probe rejects, the
 * cold rest state (n = 1, u = 0, T = T_in).  The acceptance probe (probe_steps > 0): run
 * probe_steps FP64 steps from the cold start and from the warm start; the warm start is
 * kept only where its residual is then strictly lower (a non-finite warm residual
 * rejects it).  used_warm (host array of B, may be NULL) receives 1 where the warm
 * start is kept.  Leaves the state in the FP64 buffers.  Synchronises. */
vlb_status vlb_batch_warm_start(vlb_batch* b, vlb_mlp* m, int probe_steps, int* used_warm);
/* The cold-start fallback of warm-started instances in vlb_run_to_steady: steps >= 1 of
 * the stall window (default 10000).  The report gives, per instance (host arrays of B,
 * each may be NULL), 1 while it still runs from its warm start, and the number of
 * vlb_run_to_steady steps (summed over calls since the state was replaced) at which it
 * was restarted cold (-1: never).  The stall watch also spans calls. */
vlb_status vlb_batch_set_stall_window(vlb_batch* b, long steps);
vlb_status vlb_batch_warm_report(const vlb_batch* b, int* on_warm, long* fallback_at);

/* ---- Steps without device allocation --------------------------------------------
 *
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Advances B Couette instances (the
 * descriptors of vlb_batch_create_couette) by nsteps >= 1 RK3 steps in FP64, exactly as
 * a batch created from the same descriptors would with vlb_set_state (F), vlb_step
 * (nsteps) and vlb_residual: same kernels, same default cells per run.
 *   F      device array of the state, the layout of vlb_get_state (sum over instances of
 *          2 N_R NV doubles), read and overwritten in place; owned by the caller.
 *   resid  host array of B (may be NULL): the residual of the last step (vlb_residual).
 *   hip_stream  a hipStream_t (may be NULL); the call synchronises it before returning.
 * Every other device buffer (RK stage buffers, moment sums, residual partials, tables,
 * descriptors, block lists) lives in a fixed scratch array of the library of
 * VLB_NOALLOC_SCRATCH_BYTES bytes, one per GPU, held from the first call on that GPU
 * until the process ends; the call allocates no device memory and uses no
 * allocating library routine.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other threads, other streams) race and must be serialised by the
 * caller.  Errors: VLB_EINVAL (B < 1, NULL descriptors or state, nsteps < 1, invalid
 * descriptors), VLB_EUNSTABLE (explicit dt above the limits), VLB_ENOMEM when the
 * instances need more scratch than VLB_NOALLOC_SCRATCH_BYTES (checked before any device
 * work), VLB_ENONFINITE (non-finite residual), VLB_EDEVICE. */
#define VLB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
vlb_status vlb_couette_step_noalloc(int B, const vlb_couette_desc* descs, double* F, long nsteps, double* resid,
                                    void* hip_stream);

/* ---- Expanding channel (Sec. VI) ------------------------------------------------
 *
 * A 2-D channel with walls at x = +-(1 + phi(y)), 1 + phi(xi) = 1 + (r - 1)(1 +
 * tanh(4 xi / L - 2)) / 2 (half-width 1 upstream, r downstream: the tanh wall of Eq.
 * canalie_phi rescaled to these asymptotes), in the coordinates lambda = x / (1 + phi)
 * in [-1, 1] and xi = y in [xi_in, xi_out], with the orthonormal triad of Sec. VI.A so
 * that p^lambda is normal to both walls.  N_lambda x N_xi equal cells in (lambda, xi).
 * Diffuse walls at rest with temperature T_w at lambda = -1 and +1 (Sec. VI.C.4, both
 * walls: the full channel width); reservoir ends: populations entering through the
 * inlet (outlet) see ghost cells at the Maxwellian f_eq(n_in (n_out), 0, T_w), leaving
 * ones the nearest interior cell (the construction of Sec. VI.C.1 with the density
 * fixed).  The paper's own conditions are options: half = 1 simulates lambda in [0, 1]
 * with specular reflection at the centreline; ends = 1 makes every lambda row carry the
 * parabolic flow rate Q(lambda) = 3 Q0 / (H (1 + phi)) (1 - 4 lambda^2 / H^2), H = 2, through
 * both end faces (entering populations at f_eq(n_s, u_s, T_w), u_s the profile velocity,
 * n_s from the row balance; leaving ones extrapolated at zeroth order).
 * ax1 is the p^lambda axis and must be half range (kind 1); ax2 the p^xi axis.
 * tau_model as for the Couette instances (Sec. VI uses VLB_TAU_HYDRO, Eq. canalie_tau).
 * State of an instance: [2][N_xi][N_lambda][NV] doubles (f', f''; xi cell; lambda cell;
 * k = i * Q2 + j); the initial state is the rest Maxwellian n = 1, u = 0, T = T_w
 * (written on the device).
 * Velocity sets of at most 32 x 16 or 16 x 32 nodes (tiles of 16 x 16, at most two).
 * precision VLB_FP64 or VLB_MIXED; the mixed form keeps a second state in FP32, scaled
 * by 1/(w_i w_j), on which vlb_channel_step runs (moment, wall-flux and residual sums
 * stay FP64), and finishes vlb_channel_run_to_steady in FP64.  The state crosses this
 * interface in FP64 in both forms.  dt = 0 picks cfl / (max advective rate +
 * force-operator bound / sqrt(3)), capped at 2 tau of the rest state.  Errors:
 * VLB_EINVAL (bad descriptor, velocity set too large, a tile-kernel instance with
 * 7 N_lambda x velocities x 8 bytes of 2^32 or more, or a batch whose stage launch would
 * cover 2^32 work-items), VLB_EUNSTABLE (explicit dt above the limit), VLB_ENOMEM,
 * VLB_EDEVICE. */
typedef struct {
    int N_lambda, N_xi;
    double xi_in, xi_out;
    double r, L;
    vlb_axis ax1, ax2;
    double Kn;
    int tau_model;
    double dt, cfl;
    double n_in, n_out, T_w;
    double weno_eps;
    int half;     /* 1: the upper half lambda in [0, 1] with a specular centreline (Sec. VI.C.3) */
    int ends;     /* 0: reservoirs at n_in / n_out; 1: the flow-rate profile of Sec. VI.C.1-2 */
    double Q0;    /* ends = 1: flow rate through half of the cross-section */
    int cartesian; /* 1: the Cartesian-split form of Sec. VI.G: ax1 = p^x (across), ax2 = p^y
                    * (along), no force terms, V^lambda = (p^x - lambda a p^y)/(1 + phi) with the
                    * discrete metric a = (1 + phi)(phi_{p+1/2} - phi_{p-1/2})/dchi, V^xi = (1 + phi) p^y,
                    * walls by the sign of V^lambda at the wall face (Eq. canalie_coord_nw); the half
                    * channel mirrors p^x, flow-rate ends take the Cartesian profile velocity (0, Q).
                    * FP64 only; up to 1024 velocities. */
    double A;      /* 0: equal lambda cells; 0 < A < 1: cells equal in eta with lambda = tanh(eta)/A
                    * (Eq. canalie_stretch, the paper uses A = 0.95), refined towards the walls */
    int kernel;    /* 0: automatic; 1: velocity tiles of 16 x 16 on the matrix cores (at most two
                    * tiles; FP64 or mixed); 2: the population kernel (a block per cell, a thread per
                    * velocity, up to 1024 velocities; FP64).  Automatic picks the population kernel
                    * in FP64 for sets that fill less than half their tiles or need more than two. */
} vlb_channel_desc;
typedef struct vlb_channel vlb_channel;

vlb_status vlb_channel_create(vlb_channel** out, int B, const vlb_channel_desc* descs, int precision,
                              void* hip_stream);
vlb_status vlb_channel_destroy(vlb_channel* c);
/* Channel batch in caller-supplied device memory: vlb_channel_create_deferred builds the
 * host side only (no device allocation, no HIP call); vlb_channel_workspace_bytes gives
 * the bytes it needs; vlb_channel_bind_workspace takes a 256-byte aligned device buffer
 * of at least that size (e.g. a torch tensor's storage; the caller keeps ownership and
 * must keep it alive until vlb_channel_destroy), uploads the tables and writes the rest
 * state (synchronises).  Until a workspace is bound, every call that touches the device
 * returns VLB_ESTATE.  vlb_channel_create is the same with a library-owned allocation. */
vlb_status vlb_channel_create_deferred(vlb_channel** out, int B, const vlb_channel_desc* descs, int precision,
                                       void* hip_stream);
vlb_status vlb_channel_workspace_bytes(const vlb_channel* c, size_t* bytes);
vlb_status vlb_channel_bind_workspace(vlb_channel* c, void* dev_ptr, size_t bytes);
/* Reservoir end of instance inst (ends = 0 only; end 0 = inlet xi_in, 1 = outlet xi_out):
 * the incoming populations there become the Maxwellian at rest with density n and
 * temperature T (Sec. VI.C reservoirs; the descriptor's n_in / n_out and T_w at
 * creation).  Takes effect at the next step.  Errors: VLB_EINVAL (bad arguments or an
 * instance with flow-rate ends). */
vlb_status vlb_channel_set_open_bc(vlb_channel* c, int inst, int end, double n, double T);
/* Total particle number sum dchi dlambda n of every instance (host array of B; the per-cell
 * contents come from the device, summed on the host in cell order).  Synchronises. */
vlb_status vlb_channel_total_mass(vlb_channel* c, double* Ntot);
/* Wall-clock seconds of the last vlb_channel_run_to_steady call. */
vlb_status vlb_channel_last_run_seconds(const vlb_channel* c, double* seconds);
vlb_status vlb_channel_info(const vlb_channel* c, int inst, int* N_lambda, int* N_xi, int* NV, double* dt,
                            size_t* state_offset);
vlb_status vlb_channel_state_size(const vlb_channel* c, size_t* n_doubles);
vlb_status vlb_channel_set_state(vlb_channel* c, const double* host, size_t n);
vlb_status vlb_channel_get_state(vlb_channel* c, double* host, size_t n);
/* One instance's state ([2][N_xi][N_lambda][NV] doubles, n must match), in FP64 (a mixed
 * batch's FP32 state is converted first).  Synchronise. */
vlb_status vlb_channel_get_instance_state(vlb_channel* c, int inst, double* host, size_t n);
vlb_status vlb_channel_set_instance_state(vlb_channel* c, int inst, const double* host, size_t n);
/* Instance inst set to the local equilibrium of per-cell fields (host arrays [N_xi][N_lambda]:
 * density n > 0, velocity components u^lambda, u^xi in the cell's orthonormal triad, as
 * vlb_channel_moments returns them, temperature T > 0): f' = n g1 g2, f'' = T f' with the
 * equilibrium expansion of the stage kernels (Sec. IV.D, Eqs. feq_red, eq_gak_H,
 * eq_gak_hh), computed on the device in FP64.  The learned warm start of a channel is
 * this call on the surrogate's fields.  Vielbein instances only.  Synchronises. */
vlb_status vlb_channel_init_equilibrium(vlb_channel* c, int inst, const double* n, const double* u1,
                                        const double* u2, const double* T);
/* nsteps RK3 steps in the batch's precision (FP32 for VLB_MIXED); the last records the
 * residual (same definition as for Couette, volumes dchi dlambda).  Enqueued on the
 * stream; does not synchronise. */
vlb_status vlb_channel_step(vlb_channel* c, long nsteps);
/* Step graphs (default on): runs of more than 10 steps replay a captured HIP graph of 10
 * steps (every stage launch of the batch, per precision, captured on a private stream at
 * first use) for all but the last chunk, which runs as plain launches and records the
 * residual.  enable = 0 makes every step plain launches (bitwise the same results). */
vlb_status vlb_channel_set_graphs(vlb_channel* c, int enable);
/* nsteps RK3 steps in FP64 (moves a mixed batch's state to its FP64 buffers). */
vlb_status vlb_channel_step_fp64(vlb_channel* c, long nsteps);
/* L[F] of the current state in the current precision (host array of state size, FP64
 * populations). Synchronises. */
vlb_status vlb_channel_apply_L(vlb_channel* c, double* L, size_t n);
/* FP32 steps taken by the last vlb_channel_run_to_steady (0 for FP64 batches). */
vlb_status vlb_channel_fp32_steps(const vlb_channel* c, long* n);
vlb_status vlb_channel_residual(vlb_channel* c, double* r);
/* Per cell of instance inst ([N_xi][N_lambda] host arrays, each may be NULL): n,
 * u^lambda, u^xi, T and the particle content dchi dlambda n. */
vlb_status vlb_channel_moments(vlb_channel* c, int inst, double* n, double* u1, double* u2, double* T,
                               double* content);
/* Flow diagnostics of instance inst (Sec. VI.D, VI.F), computed on the device from the
 * FP64 state (a mixed batch's FP32 state is moved there first) into host arrays, each of
 * which may be NULL:
 *   ux, uy  [N_xi][N_lambda]  Cartesian velocity (Eq. canalie_u; y along the channel);
 *   P       [N_xi][N_lambda]  pressure n T;
 *   psi     [N_xi][N_lambda + 1] stream function on the lambda faces, rho u_y = -d psi / dx
 *           (Eq. canalie_psi) summed across each xi column with dx = (1 + phi) d lambda,
 *           zero at lambda = 0 (linear inside the middle cell for odd N_lambda);
 *   omega   [N_xi][N_lambda]  vorticity of Eq. canalie_vorti at the cell centres, first
 *           derivatives by three-point formulas (centred inside, one-sided second order on
 *           the first and last cells);
 *   Pw      [2][N_xi]         P extrapolated linearly from the two outermost cells to the
 *           lambda faces 0 (lower wall, or the centreline of the half channel) and N_lambda
 *           (upper wall).
 * Synchronises.  Errors: VLB_EINVAL (bad instance), VLB_EDEVICE. */
vlb_status vlb_channel_flow_fields(vlb_channel* c, int inst, double* ux, double* uy, double* P, double* psi,
                                   double* omega, double* Pw);
vlb_status vlb_channel_run_to_steady(vlb_channel* c, double tol, long max_steps, int check_every, long* steps,
                                     double* r);

const char* vlb_status_string(vlb_status s);
const char* vlb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VLB_H */
