/*
 * expdiag.h -- C ABI of the MI355X (gfx950) Exp-ParaDiag library.
 *
 * Solves the all-at-once space-time system of an exponential integrator for
 *     u_t = a Lap(u) - b.grad(u) - c u + N(u),   N(u) = n1 u + n2 u^2 + n3 u^3,
 * on the periodic box [0, 2pi)^dim with Fourier collocation, by the
 * alpha-circulant preconditioned fixed point (Garai & Chamakuri,
 * "Exp-ParaDiag", Sec. 3, eq. pcond-1st-order, steps (a)-(c) of eq.
 * exp_ParaDiag_steps) or by preconditioned GMRES (Sec. 3.2), with the
 * nonlinearity lagged one iteration (Sec. 6.2, eq. disc_imextype_scheme).
 *
 * Time integrators (one time step dt, A = exp(dt L)):
 *   EXPDIAG_ETD1: u_n = A u_{n-1} + dt phi1(dt L) N(u_{n-1})
 *   EXPDIAG_ETD2: u_n = A u_{n-1} + dt[(phi1+phi2) N(u_{n-1}) - phi2 N(u_{n-2})],
 *                 u_{-1} := u_0
 * For N == 0 both reduce to the paper's first-order scheme u_n = A u_{n-1}
 * (Sec. 2, eq. disc_wr).
 *   EXPDIAG_IF1:  u_n = A u_{n-1} + dt N(u_n), the implicit integrating-
 *                 factor scheme of Sec. 5 (eq. fully_discrete_nonlinear).
 *                 Each Exp-ParaDiag iteration is one inexact Newton step of
 *                 eq. newton_2 with the averaged Jacobian reduced to a
 *                 scalar: the preconditioner is Q_alpha - sigma I, sigma =
 *                 dt times the space-time mean of N'(U^k) (jacobian = 1),
 *                 of N'(u0) (jacobian = 2), or 0 (jacobian = 0: the lagged
 *                 iteration of eq. disc_imextype_scheme).  Radix FFT time
 *                 transform only; expdiag_precond_apply applies sigma = 0.
 *   EXPDIAG_EBDF2 (linear problems, N == 0): the second-order exponential
 *                 BDF of Sec. 4 (eq. 2nd_order_scheme),
 *                 u_n = 4/3 A u_{n-1} - 1/3 A^2 u_{n-2}, started from
 *                 u_1 = A u_0.  Slice 1 of a window is that fixed start; the
 *                 unknowns are u_2..u_Nt (eq. all_at_once_2ndorder), whose
 *                 residual f_2 - R v takes u_1 = A u_0 whatever slice 1
 *                 holds, and whose preconditioner is R_alpha of eq.
 *                 pcond-2nd-order on Nt - 1 time points.
 *   EXPDIAG_EBDF3 .. EXPDIAG_EBDF6 (linear problems, N == 0): the
 *                 exponential BDF of order s = 3..6 of Sec. bdfs (eqs.
 *                 3rd_order_scheme .. sixth_order_scheme),
 *                 u_n = sum_{i=1..s} beta_i A^i u_{n-i}, started from
 *                 u_m = A^m u_0, m < s.  Slices 1..s-1 of a window are
 *                 those fixed starts; the unknowns are u_s..u_Nt (eqs.
 *                 all_at_once_3rdorder .. all_at_once_6thorder), with f_s
 *                 built from u_0 and the start values, and the
 *                 preconditioner R_s^alpha (C_{i-1}^alpha = (C_0^alpha)^i,
 *                 the alpha-circulants of Sec. bdfs) on Nt - s + 1 time
 *                 points.  EBDF2 is the case s = 2.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers to float64 data owned by the caller
 *     (typically torch tensors).  They must not alias each other unless
 *     stated, and must be at least 16-byte aligned.
 *   - Physical layout: a field is n[0] x .. x n[dim-1] doubles, row-major,
 *     last index fastest, grid point x_j = 2 pi j / n.  A space-time array
 *     holds slices u_1 .. u_Nt (time t_k = k dt) back to back: slice k
 *     (1-based) starts at offset (k-1) * Ns, Ns = prod n[i].
 *   - All work is enqueued on the handle's HIP stream.  expdiag_iterate and
 *     expdiag_gmres synchronise that stream before returning; the other
 *     calls only enqueue unless a host output pointer is given.
 *   - A handle owns all of its device workspace, allocated once by
 *     expdiag_create and released by expdiag_destroy; no other call
 *     allocates.  A handle must not be used by two threads at once.
 *   - Return value: EXPDIAG_OK, EXPDIAG_NOT_CONVERGED (> 0, outputs valid),
 *     or a negative error code; expdiag_strerror names it and
 *     expdiag_last_error gives the handle's last detailed message.  No C++
 *     exception crosses this boundary.
 */
#ifndef EXPDIAG_H
#define EXPDIAG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXPDIAG_OK 0
#define EXPDIAG_NOT_CONVERGED 1
#define EXPDIAG_EINVAL (-1)
#define EXPDIAG_ENOMEM (-2)
#define EXPDIAG_EHIP (-3)
#define EXPDIAG_EDIVERGED (-4)
#define EXPDIAG_EUNSUPPORTED (-5)

#define EXPDIAG_ETD1 1
#define EXPDIAG_ETD2 2
#define EXPDIAG_EBDF2 3
#define EXPDIAG_IF1 4
#define EXPDIAG_EBDF3 5
#define EXPDIAG_EBDF4 6
#define EXPDIAG_EBDF5 7
#define EXPDIAG_EBDF6 8

#define EXPDIAG_FP64 0
#define EXPDIAG_MIXED 1

typedef struct expdiag_ctx* expdiag_t;

/* Periodic grid on [0, 2pi)^dim; n[i] a power of two, 4 <= n[i] <= 4096
 * (n[dim-1] >= 4).  Entries n[dim..2] are ignored. */
typedef struct {
  int dim;
  int n[3];
} expdiag_grid;

/* u_t = a Lap(u) - b.grad(u) - c u + n1 u + n2 u^2 + n3 u^3.  The linear
 * operator is L = a Lap - c of Sec. 1 (eq. model_problem_linear) plus the
 * advection term of the remark after Theorem thm_gmres22 (periodic, so
 * diagonal in Fourier space with the complex symbol
 * -a|k|^2 - c - i b.k'; k' is the wavenumber except 0 at an axis's Nyquist
 * index, so real fields stay real); a >= 0, c >= 0, b finite (b[i] is the
 * velocity along axis i; entries past dim are ignored).
 * Complex state (complex_state = 1, linear problems only): the coefficients
 * become a + i a_im and c + i c_im (the Schroedinger equation of Sec. 6 has
 * a = i), and every physical array (u0, U, R, S) holds complex values,
 * interleaved (re, im) doubles: a field is Ns complex numbers, a window
 * Nt * Ns.  Nonzero a_im or c_im need complex_state = 1 (the operator no
 * longer maps real fields to real fields).  GMRES then treats real and
 * imaginary parts as one real vector (inner product Re(x^H y)).  The server
 * does not take complex-state requests (EUNSUPPORTED).
 * jacobian: EXPDIAG_IF1 only (0, 1 or 2; see the scheme list above).
 * precision: EXPDIAG_FP64, or EXPDIAG_MIXED (fp32 spatial FFTs and
 * nonlinearity in a bulk phase, fp64 residual and iterate afterwards; the
 * time transform is always fp64).
 * gmres_restart: Krylov space size reserved at create for expdiag_gmres
 * (0 = no GMRES workspace). */
typedef struct {
  double a, c, n1, n2, n3;
  int precision;
  int gmres_restart;
  double b[3];
  double a_im, c_im;
  int complex_state;
  int jacobian;
} expdiag_problem;

/* Build a handle: spectral symbols E = exp(dt mu), dt phi1(dt mu),
 * dt phi2(dt mu) with mu = -a|k|^2 - c, the time tables
 * gamma_l = alpha^{l/Nt} (Gamma_alpha) and lambda_m = alpha^{1/Nt}
 * e^{2 pi i m/Nt} (eigenvalues of C_0^alpha, Sec. 2), twiddles, and all
 * device workspace (size given by expdiag_footprint_bytes).
 *   g        grid (host pointer)
 *   Nt       number of time steps in the window, power of two, 2..512.
 *            An order-s exponential BDF (EBDF2..EBDF6) transforms the
 *            Nt - s + 1 unknown slices: Nt - s + 1 a power of two, 2..512,
 *            takes the radix FFT; otherwise Nt must be a power of two in
 *            8..128 and takes the dense transform
 *   dt       time step (> 0); the window is T = Nt dt
 *   alpha    circulant parameter, 0 < alpha < 1
 *   scheme   EXPDIAG_ETD1, EXPDIAG_ETD2, EXPDIAG_IF1, or EXPDIAG_EBDF2 ..
 *            EXPDIAG_EBDF6 (linear problems only; EUNSUPPORTED otherwise)
 *   p        PDE coefficients and options (host pointer)
 *   hip_stream  hipStream_t to enqueue on (NULL = default stream)
 *   out      receives the handle
 * Errors: EINVAL (bad argument), EUNSUPPORTED (size not supported), ENOMEM,
 * EHIP. */
int expdiag_create(const expdiag_grid* g, int Nt, double dt, double alpha,
                   int scheme, const expdiag_problem* p, void* hip_stream,
                   expdiag_t* out);

/* Release a handle and its workspace (NULL is accepted). */
int expdiag_destroy(expdiag_t h);

/* Replace the stream the handle enqueues on (waits for the work already
 * enqueued on the old one). */
int expdiag_set_stream(expdiag_t h, void* hip_stream);

/* Device bytes a handle with these parameters allocates (for admission
 * control); 0 on invalid arguments. */
size_t expdiag_footprint_bytes(const expdiag_grid* g, int Nt, int scheme,
                               int precision, int gmres_restart);

/* All-at-once residual R = f + G(U) - Q U (right-hand side of eq.
 * pcond-1st-order, with Q = I - C_0 (x) A and f = (A u0 + dt phi1 N(u0),
 * 0, .., 0)); slice n of R is A u_{n-1} + G_n - u_n with u_0 = u0.
 * EBDF2: slice 1 is A u0 - u_1, slices 2..Nt are f_2 - R v (eq.
 * all_at_once_2ndorder) with v = (u_2..u_Nt) and u_1 := A u0 in f_2;
 * EBDF3..6 likewise: slice m < s is A^m u0 - u_m, slices s..Nt are
 * f_s - R_s v with u_m := A^m u0 in f_s.
 *   u0    Ns doubles (device)     U, R   Nt*Ns doubles (device, distinct)
 *   rnorm if non-NULL, host pointer receiving ||R||_2 (the call then
 *         synchronises); if NULL the call only enqueues. */
int expdiag_residual(expdiag_t h, const double* u0, const double* U,
                     double* R, double* rnorm);

/* S = Q_alpha^{-1} R by the three steps of Sec. 3 (eq. exp_ParaDiag_steps):
 * (a) alpha-scaled forward time transform, (b) Nt independent shifted
 * solves (I - lambda_m A)^{-1}, pointwise in Fourier space, (c) inverse
 * time transform.  R and S are Nt*Ns doubles (device); S may equal R.
 * EBDF2: slice 1 is copied, slices 2..Nt get R_alpha^{-1} by the steps of
 * eq. exp_ParaDiag_steps_2ndorder (shifted solves
 * (I - 4/3 lambda_0 A + 1/3 lambda_1 A^2)^{-1}) on Nt - 1 points; EBDF3..6:
 * slices 1..s-1 copied, slices s..Nt get (R_s^alpha)^{-1} with shifted
 * solves (I - sum_i beta_i lambda_0^i A^i)^{-1} on Nt - s + 1 points.
 * Enqueue only. */
int expdiag_precond_apply(expdiag_t h, const double* R, double* S);

/* Preconditioned fixed point u^{k+1} = u^k + Q_alpha^{-1}(f + G(u^k) - Q u^k)
 * (eq. pcond-1st-order; nonlinear term lagged as in Sec. 6.2); for EBDF2
 * v^{k+1} = v^k + R_alpha^{-1}(f_2 - R v^k) (eq. pcond-2nd-order), slice 1
 * being set to A u0, and for EBDF3..6 the same with R_s, slices m < s set
 * to A^m u0.
 *   u0        initial condition, Ns doubles (device)
 *   U         in: initial iterate (zeros in the paper's experiments),
 *             out: final iterate; Nt*Ns doubles (device)
 *   max_iter  iteration cap (1..4096)
 *   tol       stop when ||S^k||_2 <= tol ||U^{k+1}||_2
 *   iters     (host, nullable) iterations performed
 *   rel_update (host, nullable) last ||S^k|| / ||U^{k+1}||
 * Returns OK, NOT_CONVERGED (max_iter reached), or EDIVERGED (non-finite
 * residual).  Synchronises the stream. */
int expdiag_iterate(expdiag_t h, const double* u0, double* U, int max_iter,
                    double tol, int* iters, double* rel_update);

/* Left-preconditioned GMRES(restart) (Sec. 3.2, Theorem thm_gmres1's
 * system Q_alpha^{-1} Q u = Q_alpha^{-1} f) for linear problems (EBDF2:
 * R_alpha^{-1} R v = R_alpha^{-1} f_2 of Sec. 4.2, slice 1 set to A u0
 * first; EBDF3..6: the GMRES preconditioners of Sec. bdfs, slices m < s
 * set to A^m u0 first); for
 * nonlinear problems, Newton's method on R(U) = 0 whose correction
 * equations (Q - G'(U)) d = R(U) are solved by the same preconditioned
 * GMRES with Eisenstat and Walker's forcing terms (choice 2: eta_0 = 0.1,
 * eta_k = 0.9 (||R_k|| / ||R_{k-1}||)^2 capped at 0.1, their safeguard,
 * and eta_k >= tol ||R_0|| / (2 ||R_k||)).
 *   restart   Krylov space size, 1 <= restart <= gmres_restart of create
 *   max_iter  cap on total GMRES iterations
 *   tol       linear: ||Q_alpha^{-1}(f - QU)|| <= tol ||Q_alpha^{-1} f||;
 *             nonlinear: ||R(U)|| <= tol ||R(0)||
 *   iters     (host, nullable) total GMRES iterations (linear) or
 *             Newton steps * 1000 + GMRES iterations (nonlinear)
 *   rel_resid (host, nullable) final relative residual
 * U: in initial guess, out solution.  Synchronises the stream. */
int expdiag_gmres(expdiag_t h, const double* u0, double* U, int restart,
                  int max_iter, double tol, int* iters, double* rel_resid);

/* The operator Newton's correction equation applies, preconditioned as
 * expdiag_gmres applies it: W = Q_alpha^{-1} (Q - G'(U)) V, with G'(U) the
 * derivative of the lagged nonlinear term at the iterate U (u_0 fixed;
 * Sec. 5, eq. newton_2, applied to the all-at-once system of eq.
 * all_at_once_1storder).  ETD1: slice n of G'(U)V is
 * dt phi1(dt L) [N'(u_{n-1}) v_{n-1}]; ETD2: dt[(phi1+phi2) N'(u_{n-1})
 * v_{n-1} - phi2 N'(u_{n-2}) v_{n-2}] with v_0 = v_{-1} = 0.  For linear
 * problems W = Q_alpha^{-1} Q V, GMRES's operator.  Mixed precision (d >=
 * 2): the products N'(u) v and their spatial FFTs run in fp32, as in the
 * Newton loop.
 *   u0      Ns doubles (device)
 *   U, V    Nt*Ns doubles (device): linearisation point and direction
 *   W       Nt*Ns doubles (device), distinct from U and V
 * Needs a handle created with gmres_restart >= 1 (it works in the Krylov
 * workspace; EINVAL otherwise).  Overwrites the handle's iterate state.
 * Enqueue only. */
int expdiag_newton_apply(expdiag_t h, const double* u0, const double* U,
                         const double* V, double* W);

/* Preconditioned BiCGStab (the bracketed timings of Table cpu_time_combined;
 * van der Vorst's method, shadow residual r^_0 = r_0) on the same
 * left-preconditioned system as expdiag_gmres, with the same Newton outer
 * loop for nonlinear problems (BiCGStab as the inner solver, same forcing
 * term).  Each iteration applies the preconditioned operator twice; the
 * scalars stay on the device and the call synchronises once per iteration.
 * Needs a handle created with gmres_restart >= 5 (it uses six vectors of
 * that Krylov workspace); EINVAL otherwise.
 *   max_iter  cap on total BiCGStab iterations
 *   tol       as expdiag_gmres (an iteration also ends the run when its
 *             intermediate residual s already meets it)
 *   iters, rel_resid  as expdiag_gmres
 * U: in initial guess, out solution.  Synchronises the stream. */
int expdiag_bicgstab(expdiag_t h, const double* u0, double* U, int max_iter,
                     double tol, int* iters, double* rel_resid);

/* Kernel-class timing.  While enabled (mask != 0) every launch's
 * algorithmic bytes (the data it must read and write once) and count are
 * accounted per class, and launches of the classes whose bit is set in
 * mask are bracketed by HIP events recorded on the handle's stream (those
 * solves run as plain launches rather than a graph replay).  Classes: 0
 * column FFT, 1 row FFT / nonlinearity, 2 pass B (residual + time
 * transform + shifted solve + update), 3 reductions, 4 Krylov vector
 * kernels.  read() synchronises and returns per class (host arrays of
 * nclass entries; all but ms nullable): milliseconds summed over the timed
 * launches, launches, bytes, and timed launches, since enable. */
int expdiag_profile_enable(expdiag_t h, int mask);
int expdiag_profile_read(expdiag_t h, double* ms, long* launches,
                         double* bytes, long* timed, int nclass);

/* Choose between replaying the captured hipGraph of one iteration (on) and
 * launching the same kernels one by one (off, the default: on MI355X the
 * replay measured slower at every iterate size). */
int expdiag_set_graph(expdiag_t h, int on);

/* Start this handle's solves (expdiag_iterate, expdiag_gmres,
 * expdiag_bicgstab) from the all-zero space-time iterate whatever U holds
 * (on), or from U as passed (off, the default).  With it
 * on, U is output only: its contents on entry are not read, and the forward
 * spatial transform of the guess, which would be zero, is replaced by
 * clearing the spectral iterate the solve starts from (for a mixed-precision
 * fixed-point solve that starts in the fp32 bulk phase, the fp32 copy; the
 * fp64 iterate is written before it is read); for nonlinear ETD1/ETD2
 * fixed-point solves the first iteration's nonlinear term N(0) = 0 is
 * cleared likewise and its spatial transforms are skipped.  Results equal those of a solve from a
 * zeroed U bit for bit.  EINVAL for a null handle. */
int expdiag_set_zero_guess(expdiag_t h, int on);

/* Time transform of steps (a) and (c): 0 = radix-8/4/2 FFT along time in
 * registers and LDS (any Nt), 1 = dense complex Nt x Nt GEMM on FP64 MFMA
 * (8 <= Nt <= 128).  Both compute the same operator; results agree to
 * rounding.  set() rebuilds the handle's plan (EUNSUPPORTED if the variant
 * does not cover Nt; an EBDF handle has the one variant its Nt - s + 1
 * points allow); get() returns the current one. */
int expdiag_set_time_variant(expdiag_t h, int variant);
int expdiag_get_time_variant(expdiag_t h);

/* Autotuner: times, on this handle's shape (its own buffers and stream),
 * both time transforms of pass B (20 preconditioner applies each after
 * warm-up) and both widths of the pass-A column workgroups (C or 2C
 * columns; 10 launches of the plan's column stages each), keeps the faster
 * of each (an alternative to the default must win by 2%) and applies them.
 * Decisions are kept in memory for the process and, when cache_path is
 * non-NULL, in that JSON file under the key
 * gfx950/d<d>/<n0>x<n1>x<n2>/Nt<Nt>/<fp64|mixed>; a known shape is not
 * measured again.  variant, us_fft, us_dense (host, nullable) receive the
 * time-transform choice and its per-launch times (us_dense = -1 when not
 * applicable).  EBDF and IF1 handles keep their one time transform (timed;
 * the other time is -1) and are not cached. */
int expdiag_autotune(expdiag_t h, const char* cache_path, int* variant,
                     double* us_fft, double* us_dense);

/* The handle's choices: time transform (0 radix FFT, 1 dense on MFMA; as
 * expdiag_set_time_variant) and pass-A column width (0: C, 1: 2C columns
 * per workgroup; the same transforms, bit for bit).  set() rebuilds the
 * handle's plan; EINVAL / EUNSUPPORTED as expdiag_set_time_variant. */
int expdiag_set_tuning(expdiag_t h, int time_variant, int col_wide);
int expdiag_get_tuning(expdiag_t h, int* time_variant, int* col_wide);

/* ---- Batching: many independent instances in one iteration plan ------
 * Groups `count` handles (any grids, Nt, coefficients, alpha, precision;
 * each keeps its own workspace and stays owned by the caller) so that one
 * fixed-point iteration of all of them is one launch per kernel signature,
 * captured as one hipGraph.  Every instance has its own control block:
 * converged instances drop out, mixed-precision instances switch to the
 * fp64 residual independently, and each result is the one its handle gives
 * alone (same kernels, same per-instance reduction order).  The handles must
 * not be used concurrently outside the batch.  While profiling is enabled on
 * the batch's first handle (expdiag_profile_enable), the batch's iteration
 * launches are accounted in that handle's kernel-class profile. */
typedef struct expdiag_batch* expdiag_batch_t;
int expdiag_batch_create(const expdiag_t* handles, int count,
                         void* hip_stream, expdiag_batch_t* out);
int expdiag_batch_destroy(expdiag_batch_t b);
/* Solve every instance by the fixed point of expdiag_iterate.
 *   u0s[i], Us[i]  device pointers of instance i (as in expdiag_iterate)
 *   iters, rel_update, status  host arrays of count entries (nullable):
 *   per-instance iterations, last ||S||/||U||, and return code.
 * Returns the worst per-instance code.  Synchronises the stream. */
int expdiag_batch_iterate(expdiag_batch_t b, const double* const* u0s,
                          double* const* Us, int max_iter, double tol,
                          int* iters, double* rel_update, int* status);
/* The same with a cap and a tolerance per instance: instance i stops after
 * max_iters[i] iterations (1..4096) or once ||S^k|| <= tols[i] ||U^{k+1}||
 * (tols[i] >= 0; 0 runs exactly max_iters[i] iterations).  max_iters and
 * tols are host arrays of count entries; the other arguments and the
 * return value are those of expdiag_batch_iterate. */
int expdiag_batch_iterate_each(expdiag_batch_t b, const double* const* u0s,
                               double* const* Us, const int* max_iters,
                               const double* tols, int* iters,
                               double* rel_update, int* status);
const char* expdiag_batch_last_error(expdiag_batch_t b);
/* Tune a batch: every distinct shape among its handles by expdiag_autotune
 * (once per shape; the decision is applied to every handle of the shape),
 * then the batch's plan rebuilt and captured, and three batched iterations
 * timed as graph replays and three as plain launches on the given inputs
 * (u0s, Us as in expdiag_batch_iterate; Us is read, not written); the
 * faster (replay must win by 2%) is kept for the batch's solves.
 *   shapes      (host, nullable) distinct shapes tuned
 *   graph_used  (host, nullable) 1 if iterations replay the graph
 *   ms_graph, ms_launch (host, nullable) ms per batched iteration each way
 *               (ms_graph = -1 if the capture failed)
 * Synchronises the stream. */
int expdiag_batch_autotune(expdiag_batch_t b, const double* const* u0s,
                           double* const* Us, const char* cache_path,
                           int* shapes, int* graph_used, double* ms_graph,
                           double* ms_launch);
/* 1 if the batch's iterations replay its captured graph, else 0. */
int expdiag_batch_graph(expdiag_batch_t b);

/* expdiag_set_zero_guess for every later solve of a batch
 * (expdiag_batch_iterate, expdiag_batch_iterate_each): Us are output only
 * and each instance starts from the all-zero iterate; the handles' own
 * setting is neither used nor changed.  EINVAL for a null batch. */
int expdiag_batch_set_zero_guess(expdiag_batch_t b, int on);

/* ---- Serving: continuous batching of solve requests -------------------
 * A server owns a host thread that admits submitted requests in arrival
 * order while the sum of their device footprints (expdiag_footprint_bytes)
 * stays within hbm_budget and fewer than max_active are in flight, keeps
 * each admitted solve's space-time state on the device, runs all admitted
 * solves together (the batch plan above, rebuilt when membership changes),
 * and retires each as it converges.  Requests arriving while others run
 * join at the next iteration chunk.  Should building the launch plan or
 * running a chunk fail (EHIP), nothing more is launched for that set:
 * every active and pending request is reported by poll with status
 * EXPDIAG_EHIP, their handles are released, and later submissions start
 * afresh.  (Setting the environment variable EXPDIAG_FAIL_PLAN_UPLOAD makes
 * every plan upload fail, as an out-of-memory upload would, for tests of
 * this path.) */
typedef struct expdiag_server* expdiag_server_t;
typedef struct {
  long long id;
  int status;         /* expdiag_iterate's return code for this request */
  int iters;
  double rel_update;
  double t_submit, t_admit, t_done;  /* seconds since server creation */
} expdiag_result;
int expdiag_server_create(size_t hbm_budget, int max_active,
                          void* hip_stream, expdiag_server_t* out);
/* Queue one solve; u0 (Ns doubles) and U (Nt*Ns doubles, in: initial
 * iterate, out: result) are device pointers that must stay valid, and U
 * untouched by the caller, until the request is reported by poll. */
int expdiag_server_submit(expdiag_server_t s, const expdiag_grid* g, int Nt,
                          double dt, double alpha, int scheme,
                          const expdiag_problem* p, const double* u0,
                          double* U, int max_iter, double tol,
                          long long* id);
/* Move up to cap finished results into out (host array); *n receives the
 * count, *outstanding (nullable) the requests not yet reported. */
int expdiag_server_poll(expdiag_server_t s, expdiag_result* out, int cap,
                        int* n, int* outstanding);
int expdiag_server_stats(expdiag_server_t s, size_t* bytes_in_use,
                         int* active, int* pending, double* busy_seconds);
/* Tune the handles of requests admitted from now on by their shape
 * (expdiag_autotune with cache_path, nullable; each shape is measured once
 * per process). */
int expdiag_server_autotune(expdiag_server_t s, const char* cache_path);
/* Finish every queued request, then stop the thread and free. */
int expdiag_server_destroy(expdiag_server_t s);

/* ---- No device allocation ---------------------------------------------
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of expdiag_create + expdiag_iterate + expdiag_destroy in one call, with
 * every device buffer a handle would own and the launch plan's tables
 * carved from one library-owned device workspace of 160 MiB per GPU
 * (allocated when the library is loaded, held until the process ends, the
 * address looked up once per device).  It calls no hipMalloc, hipFree or
 * hipHostMalloc.  Arguments as expdiag_create (g, Nt, dt, alpha, scheme, p
 * with gmres_restart = 0, hip_stream) and expdiag_iterate (u0, U,
 * max_iter, tol, iters, rel_update); results equal those of that pair.
 * A problem whose buffers do not fit (about 136 MB for 256^2 x 64 in mixed
 * precision, the largest 2D case that fits) is refused with EINVAL before
 * the device is touched.  The workspace keeps the last call's contents and
 * is shared by every call on a device: calls on one device are serialised
 * by a lock and each synchronises its stream before returning, so calls do
 * not overlap on a device; a caller enqueueing other work on that stream
 * must not expect it to run concurrently with this call.  Errors: as
 * expdiag_create and expdiag_iterate; expdiag_last_error(NULL) gives the
 * message. */
int expdiag_iterate_noalloc(const expdiag_grid* g, int Nt, double dt,
                            double alpha, int scheme,
                            const expdiag_problem* p, void* hip_stream,
                            const double* u0, double* U, int max_iter,
                            double tol, int* iters, double* rel_update);

/* Static description of an error code. */
const char* expdiag_strerror(int code);

/* Detailed message of the handle's last failure ("" if none). */
const char* expdiag_last_error(expdiag_t h);

#ifdef __cplusplus
}
#endif
#endif /* EXPDIAG_H */
