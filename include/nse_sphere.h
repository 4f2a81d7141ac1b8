/*
 * nse_sphere.h -- C ABI of the MI355X (gfx950) implementation of the
 * pseudospectral quadrature method for the incompressible Navier-Stokes
 * equations on the rotating unit sphere (Ganesh, Le Gia, Sloan).
 *
 * The problem (Section 4, eqs. (app_weak_form), (app1_weak_form), (ode)):
 * find u_N(t) = sum_{l=1..N, |m|<=l} alpha[l,m](t) Z[l,m] with
 *     d alpha/dt = f - nu lambda_l alpha - n(alpha),
 *     n[l,m] = (B(u_N,u_N) + C u_N, Z[l,m])_M,            lambda_l = l(l+1),
 * where Z[l,m] = lambda_l^(-1/2) Curl Y[l,m] (eq. (stok_eig)), B is the
 * advection (eqs. (B), (short_nonlin1)), C the Coriolis operator (eq. (C)) and
 * (.,.)_M the Gauss-rectangle discrete inner product (eqs. (quadrule),
 * (disc_ip)) on nlat = M/2 Gauss-Legendre latitudes x M equispaced longitudes.
 *
 * Coefficient storage (every "state" array below):
 *   complex128, interleaved (re, im) doubles, one block per member, members in
 *   the order given to nse_sphere_init. Inside a member of truncation N the
 *   slot of (l, m), 0 <= m <= l <= N, is  m*(2N+3-m)/2 + (l-m)  (m-major), so a
 *   member holds nse_coeff_count(N) = (N+1)(N+2)/2 complex values. Negative
 *   orders are implied by alpha[l,-m] = (-1)^m conj(alpha[l,m]) (real field).
 *   On input the (0,0) slot and the imaginary parts of m = 0 slots must be 0;
 *   on output they are 0.
 *
 * Memory and streams:
 *   Every array argument of a compute call is a DEVICE pointer (e.g. a torch
 *   tensor's data_ptr) owned by the caller, which keeps it alive until the work
 *   enqueued on the context's stream has completed. The library owns its
 *   tables and workspaces from nse_sphere_init to nse_sphere_destroy and never
 *   frees caller memory. All work is enqueued on the context's HIP stream;
 *   calls return before the GPU finishes (use nse_sync or the stream).
 *
 * Errors:
 *   Argument checks are synchronous: on failure a call returns NSE_ERR_ARG (or
 *   NSE_ERR_UNSUPPORTED), enqueues nothing and records a message readable with
 *   nse_last_error. HIP failures return NSE_ERR_HIP from the call that observes
 *   them (launch errors) or from nse_sync (asynchronous errors). A context is
 *   not thread-safe; separate contexts are independent.
 */
#ifndef NSE_SPHERE_H
#define NSE_SPHERE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nse_ctx nse_ctx; /* opaque, library-owned */

typedef enum {
  NSE_OK = 0,
  NSE_ERR_ARG = 1,         /* invalid argument; nothing enqueued              */
  NSE_ERR_ALLOC = 2,       /* device or host allocation failed                */
  NSE_ERR_HIP = 3,         /* a HIP runtime call or kernel launch failed      */
  NSE_ERR_UNSUPPORTED = 4, /* valid request this build does not implement     */
  NSE_ERR_NONFINITE = 5,   /* NaN/Inf detected (NSE_FLAG_CHECK_FINITE)        */
  NSE_ERR_STATE = 6        /* call not valid in the context's current state   */
} nse_status;

/* Precision of the Legendre contractions (the direct synthesis and analysis sums
 * of Section 4.2). The quadrature weights, FFTs, grid products and the viscous
 * update always run in FP64, and so do the Legendre values: FP64 and FP32
 * continue the three-term recurrence in FP64 registers from FP64 seed rows;
 * BF16X3 reads the FP64 table rounded once to FP32. */
enum {
  NSE_PREC_FP64 = 0,  /* FP64 products, FP64 accumulation                      */
  NSE_PREC_FP32 = 1,  /* values and coefficients rounded to FP32, FP32 products
                         and per-wave accumulation, FP64 cross-wave sums      */
  NSE_PREC_BF16X3 = 2 /* operands split into three bf16 pieces, MFMA, FP32 acc */
};

enum {
  NSE_FLAG_GRAPH = 1,       /* replay nse_step through a captured hipGraph      */
  NSE_FLAG_AUTOTUNE = 2,    /* time the member-block sizes of every FP64 group
                               with >= 2 members at init and keep the fastest */
  NSE_FLAG_CHECK_FINITE = 4 /* flag NaN/Inf in the state; nse_sync reports it   */
};

/* One ensemble member: truncation N >= 1, latitudes nlat (0 = the smallest nlat
 * with M = 2 nlat >= 3N + 2, eq. (M_choice), whose M factors into 2, 3 and 5),
 * viscosity nu >= 0. */
typedef struct {
  int32_t N;
  int32_t nlat;
  double nu;
} nse_member;

/* Shared parameters: rotation Omega (eq. (C)), step h, NDF order p in 1..5 of
 * eq. (ode_disc) (kappa_p as printed in Section 4.2), fixed-point sweeps of
 * the implicit step (1 = nonlinear term at the extrapolated predictor), the
 * contraction precision and NSE_FLAG_* flags. */
typedef struct {
  double omega;
  double dt;
  int32_t order;
  int32_t newton_iters;
  int32_t precision;
  uint32_t flags;
} nse_params;

/* Creates a context: computes the Gauss-Legendre rule (eq. (quadrule)) on the
 * host, the normalised Legendre tables Pbar[l,m](mu_p), l <= N+1, in FP64 on
 * the GPU (eq. (sph_har)), FFT twiddles and workspaces. `hip_stream` is a
 * hipStream_t (NULL = default stream). Returns NSE_ERR_ARG for n_members < 1,
 * N < 1, 2*nlat < 3N+2, nu < 0, order outside 1..5, newton_iters < 1, an
 * unknown precision or flag; NSE_ERR_UNSUPPORTED for a grid whose M has a prime
 * factor other than 2, 3, 5 or M > 1536. *out is NULL on failure. */
nse_status nse_sphere_init(const nse_member* members, int32_t n_members,
                           const nse_params* params, void* hip_stream,
                           nse_ctx** out);

/* Waits for the context's stream, frees everything it owns. NULL is a no-op. */
nse_status nse_sphere_destroy(nse_ctx* ctx);

/* Member blocking of a truncation group (members sharing N and nlat). In FP64
 * a group with several members runs its Legendre synthesis and analysis as
 * FP64 MFMA products in which one pass over the table serves a block of
 * members (the same sums as Section 4.2; the table entries are reused as the
 * rows of a matrix product whose columns are the members' panels or ring
 * spectra). synth_block and anal_block are 0 (one member per workgroup, the
 * single-member kernels) or 2, 4, 8. The default for FP64 groups of >= 2
 * members is the largest power of two <= min(members, 4) for the synthesis
 * and <= min(members, 8) for the analysis, or what NSE_FLAG_AUTOTUNE measured. `member` selects the group by any of its
 * members. Other precisions always use the single-member kernels. Setting
 * drops captured graphs. NSE_ERR_ARG for an unknown block size or member, or
 * for non-zero blocks on a group of one member or of another precision. */
nse_status nse_get_member_blocks(const nse_ctx* ctx, int32_t member,
                                 int32_t* synth_block, int32_t* anal_block);
nse_status nse_set_member_blocks(nse_ctx* ctx, int32_t member,
                                 int32_t synth_block, int32_t anal_block);

/* Rebinds the context to another hipStream_t (captured graphs are dropped). */
nse_status nse_set_stream(nse_ctx* ctx, void* hip_stream);

/* (N+1)(N+2)/2, or -1 for N < 0. */
int64_t nse_coeff_count(int32_t N);

/* Complex slots of one full state (sum over members), -1 for NULL. */
int64_t nse_state_count(const nse_ctx* ctx);

/* Grid of member `member`: writes nlat (and M = 2 nlat) through the int
 * pointers and, if non-NULL, the nodes mu_p (descending, north first) and
 * weights w_p into HOST arrays of nlat doubles. */
nse_status nse_member_grid(const nse_ctx* ctx, int32_t member, int32_t* nlat,
                           double* mu_host, double* w_host);

/* n = (B(u,u) + C u, Z[l,m])_M for every member (eqs. (app1_weak_form),
 * (Coriolis_ZLm), (eval_nonlin)), computed by synthesis onto the grid
 * (Legendre contraction per order m, inverse real FFT per latitude), the
 * product u . Grad(zeta + 2 Omega cos theta) on the grid, and quadrature
 * analysis (forward FFT, weighted Legendre contraction).
 * alpha, n_out: device state arrays (may not alias). */
nse_status nse_nonlinear(nse_ctx* ctx, const double* alpha, double* n_out);

/* Advances `nsteps` steps of the NDF_p formula (eq. (ode_disc)) with the
 * nonlinear term at the predictor and the Stokes term nu lambda_l (eq.
 * (stok_eig)) implicit and diagonal. hist: device array [order+1][state]
 * (hist[0] = newest state, hist[j] = the state j steps earlier), updated in
 * place and rotated. forcing: device state array of f[l,m] = (f, Z[l,m])_M,
 * constant over the call, or NULL for f = 0. step0: global index of the first
 * step (0 = the first step of the run); steps k < order+1 use the reduced
 * start-up order q = min(p, k+1). */
nse_status nse_step(nse_ctx* ctx, double* hist, const double* forcing,
                    int64_t step0, int32_t nsteps);

/* Vector-Jacobian product of nse_nonlinear at alpha: alpha_bar = J^T n_bar,
 * J the Jacobian of the real map (re, im) -> (re, im) on the stored doubles.
 * Device state arrays; alpha_bar is overwritten. */
nse_status nse_nonlinear_adjoint(nse_ctx* ctx, const double* alpha,
                                 const double* n_bar, double* alpha_bar);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as nse_nonlinear_adjoint (the same kernels), with the adjoint's
 * Fourier intermediates (5 + 4 field slabs of nlat x (N+1) complex values and
 * (N+1)(N+2)x4 panel cotangents per member, each group's pieces 256-byte
 * aligned) placed in a static device array of 32 MiB that the library holds on
 * every device it runs on until the process ends, instead of buffers the
 * context allocates on first use. It calls no allocator. One member up to
 * N = 255 on its default grid fits (18.4 MB); a context that needs more returns
 * NSE_ERR_ARG and enqueues nothing. The array is shared by every call on one
 * device and keeps the last call's contents (every entry a call reads it first
 * writes, so nothing needs clearing): calls that overlap on one device (other
 * streams, other contexts, other host threads) race. Arguments, layout and
 * errors as nse_nonlinear_adjoint. */
nse_status nse_nonlinear_adjoint_noalloc(nse_ctx* ctx, const double* alpha,
                                         const double* n_bar, double* alpha_bar);

/* Adjoint of one nse_step call with nsteps = 1 at global step index `step`:
 * hist is the history BEFORE that step ([order+1][state], device), hist_bar
 * holds dL/d(history after the step) on input and dL/d(history before the
 * step) on output (device, [order+1][state]). The forcing is not
 * differentiated. Requires newton_iters == 1. */
nse_status nse_step_adjoint(nse_ctx* ctx, const double* hist,
                            const double* forcing, int64_t step,
                            double* hist_bar);

/* nsteps steps of nse_step (eq. (ode_disc)) on a trajectory buffer: traj is a
 * device array of nsteps + order + 1 states; on entry traj[nsteps + j] holds
 * alpha_{step0 - j} (j = 0..order: the history of nse_step), and step
 * step0 + i (i = 0..nsteps-1) reads its history from traj[nsteps - i ..]
 * (newest first) and writes its new state to traj[nsteps - i - 1]. On return
 * traj[0] is the final state and traj[nsteps - i ..] is the history before step
 * step0 + i, as nse_step_adjoint_trajectory reads it. The results equal those
 * of nse_step (the same kernels; the new state is stored one slot lower
 * instead of rotating the history). With NSE_FLAG_GRAPH the steps with fixed
 * coefficients (index > order) replay one captured graph per (traj, forcing,
 * nsteps, step0 range). NSE_ERR_ARG for NULL traj or negative step0, nsteps. */
nse_status nse_step_trajectory(nse_ctx* ctx, double* traj, const double* forcing,
                               int64_t step0, int32_t nsteps);

/* The adjoint of nse_step_trajectory over the same traj (unchanged since):
 * hist_bar ([order+1][state], device) holds dL/d(history after step
 * step0 + nsteps - 1) on input and dL/d(history before step step0) on output,
 * the step adjoints of nse_step_adjoint applied from the last step back, each
 * reading its history from traj. Requires newton_iters == 1; hist_bar may not
 * overlap traj. With NSE_FLAG_GRAPH the fixed-coefficient steps replay one
 * captured graph per (traj, hist_bar, nsteps, step0 range). */
nse_status nse_step_adjoint_trajectory(nse_ctx* ctx, const double* traj, const double* forcing,
                                       int64_t step0, int32_t nsteps, double* hist_bar);

/* Grid values of u_theta, u_phi and zeta for every member: device array
 * [member][3][nlat][M] of doubles (latitudes north to south, longitudes
 * phi_j = 2 pi j / M). */
nse_status nse_synthesize(nse_ctx* ctx, const double* alpha, double* grid_out);

/* Discrete projection of a grid velocity field onto the divergence-free
 * basis, alpha[l,m] = (u, Z[l,m])_M (Section 3, the discrete vector inner
 * product and the orthogonal projection L_N; the initial state of the ODE is
 * obtained this way from u_0). u_grid: device array [member][2][nlat][M] of
 * doubles holding u_theta then u_phi on the grid of nse_synthesize;
 * alpha_out: device state array, overwritten (l = 0 slot and Im of m = 0
 * written as 0). For u in the span of Z[l,m], l <= N, this inverts
 * nse_synthesize exactly (up to rounding). */
nse_status nse_analyze_velocity(nse_ctx* ctx, const double* u_grid, double* alpha_out);

/* Normalised Legendre values of one member's table: writes Pbar[l,m](mu_p)
 * for l = m..N+1 and the nlat/2 northern nodes p as a device array
 * [l-m][p] of doubles. For testing the FP64 table. */
nse_status nse_legendre_values(nse_ctx* ctx, int32_t member, int32_t m,
                               double* out);

/* ---------------------------------------------------------------------------
 * Diagnostics of the experiments (Section 5.3).
 * ------------------------------------------------------------------------- */

/* Energy spectrum of every member (eq. (energy)): E(L) = sum_{|m|<=L}
 * |alpha[L,m]|^2 for L = 0..N (the stored m > 0 coefficient counts for m and
 * -m). alpha: device state; E_out: device doubles [member][N_member + 1],
 * members in order. */
nse_status nse_energy_spectrum(nse_ctx* ctx, const double* alpha, double* E_out);

/* As nse_synthesize, with the vorticity stream function of eq. (eq:vort_app),
 * Psi_N = -sum lambda^(-1/2) alpha[L,m] Y[L,m] (so that the vorticity is
 * xhat Delta Psi_N), in place of the vorticity: grid_out holds u_theta, u_phi,
 * Psi_N per member. */
nse_status nse_synthesize_psi(nse_ctx* ctx, const double* alpha, double* grid_out);

/* Approximate inertial manifold (eq. (eq:p-p)): for every member (truncation
 * N', viscosity nu > 0; Omega of the context)
 *   phi = (nu A + C)^(-1) (P_N' - P_N1) [f - B(u1, u1)],  u1 = P_N1 u,
 * with B the advection term alone, evaluated by the hot path on the member's
 * grid (exact for u1 of degree N1 <= N'), and (nu A + C) diagonal on Z[L,m]:
 * nu lambda_L - 2 i Omega m / lambda_L (eqs. (stok_eig), (Coriolis_ZLm)). The
 * paper takes N' = 2 N1. alpha_src: device coefficients of u stored at
 * truncation n_src, [member][(n_src+1)(n_src+2)/2]; only degrees <= N1 are read.
 * forcing: device state of the context (NULL = 0). phi_out: device state of the
 * context, zero at degrees <= N1. NSE_ERR_ARG for N1 outside 1..n_src or above
 * a member's N, nu <= 0, or phi_out aliasing an input. */
nse_status nse_inertial_manifold(nse_ctx* ctx, const double* alpha_src, int32_t n_src,
                                 int32_t N1, const double* forcing, double* phi_out);

/* ---------------------------------------------------------------------------
 * Adaptive time integration: the NDF_p formulas of eq. (ode_disc) (Section
 * 4.2; orders 1..5 with the kappa_p printed there), run with variable order and
 * variable step at a relative error tolerance as in the experiments of
 * Section 5 (Example 2: orders one to five, tolerance 1e-3). The state is kept
 * in backward differences D[j] = nabla^j alpha_n at the current step h; an
 * attempt of order k predicts y0 = sum_{j<=k} D[j] and iterates the corrector
 *   d = (h (f(t+h) - n(y)) - h nu lambda y0 - sum_{1<=j<=k} gamma_j D[j])
 *       / ((1 - kappa_k) gamma_k + h nu lambda),   y = y0 + d,
 * (gamma_j = sum_{i<=j} 1/i; simplified Newton with the diagonal Stokes part
 * as iteration matrix), with n from the hot path. The local error estimate is
 * (kappa_k gamma_k + 1/(k+1)) ||d||, ||v|| = max over coefficients of
 * |v| / max(|alpha_n|, |y|, atol/rtol) (complex modulus, all members of the
 * context form one system with one step). Control:
 *  - Newton: at most max_newton sweeps; from the second on, rho = ratio of
 *    successive correction norms; rho >= 0.9 fails, rho/(1-rho) * norm <=
 *    0.1 rtol converges (one sweep, max_newton = 1, always converges); a
 *    failure multiplies h by 0.3;
 *  - error failure (estimate > rtol): the first in a row multiplies h by
 *    max(0.1, 0.833 (rtol/err)^(1/(k+1))) or lowers the order if
 *    min(1, max(0.1, 0.769 (rtol/err_{k-1})^(1/k))) is larger (err_{k-1} from
 *    nabla^k alpha_{n+1}); the next ones halve h, from the third on at order 1;
 *  - after k+2 accepted steps at the same h and k, the ratios
 *    1 / max(0.1, c (err_j/rtol)^(1/(j+1))) of orders j = k (c = 1.2), k-1
 *    (1.3) and k+1 (1.4, from nabla^{k+2} alpha_{n+1}) are compared; the largest
 *    (ties: current, then lower order) is taken if it exceeds 1;
 *  - h <= hmax; a step ending within 10 % of t_end is set to end there; a new
 *    h rescales D[0..k] to the interpolating polynomial's differences at the
 *    new spacing;
 *  - first step: order 1, h = min(hmax, t_end - t0, 0.8 sqrt(rtol)/||F(t0)||)
 *    unless h0 > 0, D[1] = h F(t0, alpha0), F = f - nu lambda alpha - n.
 * ------------------------------------------------------------------------- */
typedef struct {
  double rtol;         /* relative tolerance, > 0 (the paper's: 1e-3)      */
  double atol;         /* absolute tolerance per coefficient, > 0          */
  double h0;           /* first step (0 = chosen as above)                 */
  double hmax;         /* largest step (0 = unbounded)                     */
  int32_t max_order;   /* 1..5                                            */
  int32_t max_newton;  /* corrector sweeps per attempt, 1..8              */
} nse_adaptive_params;

/* The forcing at time t is s(t) * forcing, s = fn(user, t) (1 when fn is
 * NULL). fn is called before the forcing is read for time t (once per attempt,
 * with t = t_n + h, and once by nse_adaptive_begin with t0). It may also
 * rewrite the forcing buffer and call the context's other entry points (not
 * nse_adaptive_*); work it enqueues must be on the context's stream or complete
 * before it returns. */
typedef double (*nse_forcing_fn)(void* user, double t);

/* A forcing scale the device evaluates itself (nse_adaptive_begin_scheduled):
 *   s(t) = before                                               for t <= t_on,
 *   s(t) = amp cos(omega t + phase) exp(-decay (t - t_on))      for t > t_on,
 * the switched-on, decaying oscillation of Example 2 (Section 5) as a family. */
typedef struct {
  double t_on, before, amp, omega, phase, decay;
} nse_forcing_schedule;

enum { NSE_ATTEMPT_ACCEPTED = 0, NSE_ATTEMPT_ERROR_FAIL = 1, NSE_ATTEMPT_NEWTON_FAIL = 2 };

typedef struct {
  double t;            /* start of the attempted step                     */
  double h;            /* its size                                        */
  double err;          /* error estimate (NaN after a Newton failure)     */
  int32_t order;       /* NDF order of the attempt                        */
  int32_t sweeps;      /* corrector sweeps run                            */
  int32_t outcome;     /* NSE_ATTEMPT_*                                   */
  int32_t reserved;
} nse_adaptive_record;

typedef struct {
  double t, h;         /* current time and next step                      */
  int32_t order;       /* next order                                      */
  int32_t reserved;
  int64_t accepted, error_failures, newton_failures;
  int64_t evaluations; /* nonlinear-term evaluations (hot-path chains)    */
  int64_t waits;       /* host waits (corrector norms, or attempt batches) */
  double wait_seconds; /* host time spent in those waits                  */
} nse_adaptive_stats;

/* Starts an adaptive integration at (t0, alpha0): alpha0 is a device state of
 * nse_state_count complex coefficients (copied), `forcing` a device state read
 * at every attempt (NULL = zero forcing; caller-owned, must stay valid until
 * the last nse_adaptive_advance), `fn` (may be NULL) scales or refreshes it per
 * time level. Evaluates F(t0, alpha0) once. Clears the attempt log. NSE_ERR_ARG for
 * invalid parameters (rtol or atol not > 0, h0 or hmax < 0, max_order outside
 * 1..5, max_newton outside 1..8) or NULL alpha0. */
nse_status nse_adaptive_begin(nse_ctx* ctx, const double* alpha0, double t0,
                              const nse_adaptive_params* params, const double* forcing,
                              nse_forcing_fn fn, void* user);

/* As nse_adaptive_begin with the forcing s(t) * forcing, s from `schedule`
 * (NULL: s = 1). With no host callback to call, the controller (Newton test,
 * error test, step and order choice) runs on the device after every corrector
 * sweep, and nse_adaptive_advance enqueues captured attempt sequences whose
 * kernels do nothing once the attempt has ended, waiting on the stream only
 * between batches of attempts. nse_adaptive_begin with fn = NULL takes the same
 * path; with a callback the controller runs on the host. */
nse_status nse_adaptive_begin_scheduled(nse_ctx* ctx, const double* alpha0, double t0,
                                        const nse_adaptive_params* params,
                                        const double* forcing,
                                        const nse_forcing_schedule* schedule);

/* Integrates to t_end (>= the current time), ending exactly there, and writes
 * alpha(t_end) to the device state alpha_out (may be NULL); fills *stats if
 * non-NULL. With a forcing callback (host controller) it waits on the stream
 * once per corrector sweep from the second on and once per attempt; otherwise
 * once per batch of attempts (stats->waits counts the waits either way).
 * NSE_ERR_STATE before nse_adaptive_begin or when the step falls below
 * 16 eps |t|; NSE_ERR_NONFINITE if a norm is NaN/Inf (the integration cannot
 * continue; call nse_adaptive_begin again). */
nse_status nse_adaptive_advance(nse_ctx* ctx, double t_end, double* alpha_out,
                                nse_adaptive_stats* stats);

/* Copies up to `capacity` records of the attempts since nse_adaptive_begin (in
 * order) to `out` (host) and the total number of attempts to *count. */
nse_status nse_adaptive_log(const nse_ctx* ctx, nse_adaptive_record* out, int64_t capacity,
                            int64_t* count);

/* Kernels of the hot path, for per-kernel timing. */
enum {
  NSE_KERNEL_SYNTHESIS = 0, /* Legendre synthesis of the four grid fields     */
  NSE_KERNEL_RING = 1,      /* longitude FFTs + grid product + forward FFT    */
  NSE_KERNEL_ANALYSIS = 2,  /* weighted Legendre analysis (+ step update)     */
  NSE_KERNEL_KINDS = 3
};

/* Per-kernel timing. enable = R > 0 turns it on: every kernel launch of the
 * context is then issued R times back to back between two HIP events on the
 * context stream (the event overhead is spread over the R launches), and
 * nse_step does not replay graphs. The launches are repeated on identical
 * inputs; a step's final analysis, which rotates the history in place, is
 * repeated from a saved copy of the history and redone once after the
 * events, so results are unchanged. enable = 0 turns timing off; R is at
 * most 1000. nse_profile_read waits for the stream and returns, for kernel
 * kind `kind`, the logical launches and their summed per-launch duration
 * (bracket time / R) in milliseconds since the last read or enable; it then
 * resets that kind's counters. */
nse_status nse_profile_enable(nse_ctx* ctx, int32_t enable);
nse_status nse_profile_read(nse_ctx* ctx, int32_t kind, int64_t* launches,
                            double* total_ms);

/* Blocks until the stream is idle; reports asynchronous HIP errors and, with
 * NSE_FLAG_CHECK_FINITE, NSE_ERR_NONFINITE if a step produced NaN/Inf. */
nse_status nse_sync(nse_ctx* ctx);

const char* nse_status_string(nse_status s);
const char* nse_last_error(const nse_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* NSE_SPHERE_H */
