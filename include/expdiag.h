/*
 * expdiag.h -- C ABI of the MI355X (gfx950) Exp-ParaDiag library.
 *
 * Solves the all-at-once space-time system of an exponential integrator for
 *     u_t = a Lap(u) - c u + N(u),   N(u) = n1 u + n2 u^2 + n3 u^3,
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

#define EXPDIAG_FP64 0
#define EXPDIAG_MIXED 1

typedef struct expdiag_ctx* expdiag_t;

/* Periodic grid on [0, 2pi)^dim; n[i] a power of two, 4 <= n[i] <= 1024
 * (n[dim-1] >= 4).  Entries n[dim..2] are ignored. */
typedef struct {
  int dim;
  int n[3];
} expdiag_grid;

/* u_t = a Lap(u) - c u + n1 u + n2 u^2 + n3 u^3.  The linear operator is
 * L = a Lap - c of Sec. 1 (eq. model_problem_linear); a >= 0, c >= 0.
 * precision: EXPDIAG_FP64, or EXPDIAG_MIXED (fp32 spatial FFTs and
 * nonlinearity in a bulk phase, fp64 residual and iterate afterwards; the
 * time transform is always fp64).
 * gmres_restart: Krylov space size reserved at create for expdiag_gmres
 * (0 = no GMRES workspace). */
typedef struct {
  double a, c, n1, n2, n3;
  int precision;
  int gmres_restart;
} expdiag_problem;

/* Build a handle: spectral symbols E = exp(dt mu), dt phi1(dt mu),
 * dt phi2(dt mu) with mu = -a|k|^2 - c, the time tables
 * gamma_l = alpha^{l/Nt} (Gamma_alpha) and lambda_m = alpha^{1/Nt}
 * e^{2 pi i m/Nt} (eigenvalues of C_0^alpha, Sec. 2), twiddles, and all
 * device workspace (size given by expdiag_footprint_bytes).
 *   g        grid (host pointer)
 *   Nt       number of time steps in the window, power of two, 2..512
 *   dt       time step (> 0); the window is T = Nt dt
 *   alpha    circulant parameter, 0 < alpha < 1
 *   scheme   EXPDIAG_ETD1 or EXPDIAG_ETD2
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

/* Replace the stream the handle enqueues on. */
int expdiag_set_stream(expdiag_t h, void* hip_stream);

/* Device bytes a handle with these parameters allocates (for admission
 * control); 0 on invalid arguments. */
size_t expdiag_footprint_bytes(const expdiag_grid* g, int Nt, int scheme,
                               int precision, int gmres_restart);

/* All-at-once residual R = f + G(U) - Q U (right-hand side of eq.
 * pcond-1st-order, with Q = I - C_0 (x) A and f = (A u0 + dt phi1 N(u0),
 * 0, .., 0)); slice n of R is A u_{n-1} + G_n - u_n with u_0 = u0.
 *   u0    Ns doubles (device)     U, R   Nt*Ns doubles (device, distinct)
 *   rnorm if non-NULL, host pointer receiving ||R||_2 (the call then
 *         synchronises); if NULL the call only enqueues. */
int expdiag_residual(expdiag_t h, const double* u0, const double* U,
                     double* R, double* rnorm);

/* S = Q_alpha^{-1} R by the three steps of Sec. 3 (eq. exp_ParaDiag_steps):
 * (a) alpha-scaled forward time transform, (b) Nt independent shifted
 * solves (I - lambda_m A)^{-1}, pointwise in Fourier space, (c) inverse
 * time transform.  R and S are Nt*Ns doubles (device); S may equal R.
 * Enqueue only. */
int expdiag_precond_apply(expdiag_t h, const double* R, double* S);

/* Preconditioned fixed point u^{k+1} = u^k + Q_alpha^{-1}(f + G(u^k) - Q u^k)
 * (eq. pcond-1st-order; nonlinear term lagged as in Sec. 6.2).
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
 * system Q_alpha^{-1} Q u = Q_alpha^{-1} f) for linear problems; for
 * nonlinear problems, Newton's method on R(U) = 0 whose correction
 * equations (Q - G'(U)) d = R(U) are solved by the same preconditioned
 * GMRES with forcing term min(1e-3, ||R_j|| / ||R_0||).
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

/* Kernel-class timing with HIP events recorded on the handle's stream
 * around every launch while enabled.  Classes: 0 column FFT, 1 row FFT /
 * nonlinearity, 2 pass B (residual + time transform + shifted solve +
 * update), 3 reductions, 4 Krylov vector kernels.  read() synchronises and
 * returns, per class (host arrays of nclass entries, launches and bytes
 * nullable): total milliseconds, launch counts, and algorithmic bytes (the
 * data each launch must read and write once) since enable. */
int expdiag_profile_enable(expdiag_t h, int on);
int expdiag_profile_read(expdiag_t h, double* ms, long* launches,
                         double* bytes, int nclass);

/* Static description of an error code. */
const char* expdiag_strerror(int code);

/* Detailed message of the handle's last failure ("" if none). */
const char* expdiag_last_error(expdiag_t h);

#ifdef __cplusplus
}
#endif
#endif /* EXPDIAG_H */
