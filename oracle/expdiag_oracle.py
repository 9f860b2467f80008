"""CPU FP64 reference implementation of Exp-ParaDiag -- test infrastructure only.

This module is the oracle the GPU library is checked against.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path never does.  It shares no code with the GPU library.

It is deliberately plain: numpy FP64, the paper's steps in the paper's order,
no blocking or fusion.  Library primitives used as steps: numpy's FFT (for
functions of the periodic spectral operator and for the unitary time DFT F),
numpy.linalg (dense checks).

Reference: Garai & Chamakuri, "Exp-ParaDiag: Time-Parallel Exponential
Integrators for Parabolic PDEs" (arXiv 2603.04350).  Citations below name the
section / equation of that paper.

Readings taken where the paper is silent:
  * Spatial operator: Fourier collocation on periodic [0,2pi)^d, n even,
    L = a*Lap - b.grad - c with symbol mu_k = -a|k|^2 - c - i b.k' (the
    analysis of Sec. 2-3 only needs L_h diagonalisable with spectrum in the
    closed left half plane; the advection term is the one of the remark
    after Theorem thm_gmres22).  k' is the derivative wavenumber: k, except
    0 at the Nyquist index, so that L maps real fields to real fields.
  * ETD1 = explicit exponential Euler,
        u_n = A u_{n-1} + dt*phi1(dt L) N(u_{n-1}),
    the ETD variant Sec. 5 allows; the all-at-once iteration lags the
    nonlinearity exactly as in the IMEX-type iteration of Sec. 6.2
    (eq. disc_imextype_scheme), here with the phi1-weighted term.
  * ETD2 = Cox-Matthews multistep,
        u_n = A u_{n-1} + dt[(phi1+phi2) N(u_{n-1}) - phi2 N(u_{n-2})],
    with u_{-1} := u_0 (so step 1 equals ETD1).
  * N(u) = n1 u + n2 u^2 + n3 u^3 evaluated pointwise on the grid, no
    dealiasing.
  * The fixed point is written in residual-correction form
    u^{k+1} = u^k + Q_alpha^{-1}(f + G(u^k) - Q u^k)  (eq. pcond-1st-order),
    which equals the paper's b^{k-1} form in exact arithmetic.
  * Complex coefficients a + i a_im, c + i c_im (the Schroedinger equation
    of Sec. 6 has a = i) make the state complex; such a Setup (or one with
    cstate=True) keeps every field complex and takes no real part.  GMRES
    then runs on the real and imaginary parts as one real vector (inner
    product Re(x^H y)).
  * IF1 (scheme 4, Sec. 5, eq. fully_discrete_nonlinear): u_n = A u_{n-1}
    + dt N(u_n).  The iteration is the residual-correction fixed point with
    the preconditioner Q_alpha - sigma I, sigma = dt times a scalar Jacobian
    (if1_sigma): one inexact Newton step of eq. newton_2 per Exp-ParaDiag
    iteration, with the averaged Jacobian reduced to its space-time mean so
    that step (b) stays pointwise; sigma = 0 is the lagged iteration of eq.
    disc_imextype_scheme.
  * EBDF2 (scheme 3, Sec. 4, linear problems only): the starting value is
    u_1 = A u_0, the exact exponential step (the paper leaves u_1 open).
    Space-time arrays still hold u_1..u_Nt; the unknown of the paper's
    system is v = (u_2..u_Nt), and f_2 is built from u_0 and that u_1, so
    the iteration on v does not depend on what slice 1 holds.  Slice 1's
    own residual row is A u_0 - u_1 and its preconditioner is the identity.
  * EBDF3..EBDF6 (schemes 5..8, Sec. bdfs, linear problems only): the same
    construction with start values u_j = A^j u_0, j = 1..s-1, unknowns
    v = (u_s..u_Nt) on N = Nt - s + 1 slices and C_{j-1}^alpha =
    (C_0^alpha)^j, the matrix whose alpha entries sit where the paper lists
    them for C_1..C_5 (its list names C_3 twice; the second is C_4 and the
    one called C_4 is C_5).  Step (b) then inverts
    I - sum_j beta_j lambda_{0,m}^j A^j.  The fixed point of eq.
    pcond-2nd-order carries over (the paper only runs GMRES for s >= 3).
  * BiCGStab (Table cpu_time_combined) runs on the same left-preconditioned
    system as GMRES, with the shadow residual r^_0 = r_0.

parity: every function here is pinned by tests/test_oracle_pins.py and, for
EBDF2, tests/test_oracle_ebdf2.py (closed forms, dense LU, mpmath, textbook
GMRES, convergence order, the exact spectra of Sec. 4); EBDF3..6 and
BiCGStab by tests/test_oracle_ebdf_bicgstab.py (BDF coefficients from the
backward-difference definition, exactness on A^n u_0, dense LU of the
assembled systems, matrix powers of C_0^alpha, scipy's BiCGStab).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Setup", "phi1", "phi2", "sequential", "residual", "precond_apply",
    "fixed_point", "q_apply", "qalpha_apply", "gprime_apply",
    "nonlinear_term", "gmres",
    "gmres_solve", "newton_gmres", "rel_err", "dense_operators",
    "dense_solve", "dense_newton", "time_dft", "time_idft",
    "EBDF2", "ebdf2_tables", "sequential_ebdf2", "residual_ebdf2",
    "r_apply_ebdf2", "ralpha_apply_ebdf2", "precond_apply_ebdf2",
    "gmres_solve_ebdf2", "dense_operators_ebdf2",
    "IF1", "sequential_if1", "residual_if1", "precond_apply_if1",
    "if1_sigma", "dense_newton_if1", "outer_iteration_if1",
    "EBDF3", "EBDF4", "EBDF5", "EBDF6", "EBDF_COEFFS", "ebdf_order",
    "ebdf_beta", "ebdf_tables", "sequential_ebdf", "r_apply_ebdf",
    "ralpha_apply_ebdf", "residual_ebdf", "precond_apply_ebdf",
    "gmres_solve_ebdf", "dense_operators_ebdf", "bicgstab",
    "bicgstab_solve", "newton_bicgstab",
]

EBDF2 = 3  # scheme code of the second-order exponential BDF (Sec. 4)
IF1 = 4    # scheme code of the implicit integrating-factor scheme (Sec. 5)
EBDF3, EBDF4, EBDF5, EBDF6 = 5, 6, 7, 8  # exponential BDF3..6 (Sec. bdfs)


# ---------------------------------------------------------------------------
# phi functions (exponential-integrator weights)
# ---------------------------------------------------------------------------
def _as_float(z):
    z = np.asarray(z)
    return z if np.iscomplexobj(z) else z.astype(np.float64)


def phi1(z):
    """phi1(z) = (e^z - 1)/z, phi1(0) = 1 (exponential Euler weight); real
    or complex z."""
    z = _as_float(z)
    out = np.ones_like(z)
    nz = z != 0.0
    out[nz] = np.expm1(z[nz]) / z[nz]
    return out


def phi2(z):
    """phi2(z) = (e^z - 1 - z)/z^2, phi2(0) = 1/2.

    For |z| < 1 the direct formula cancels, so the Taylor series
    sum_{j>=0} z^j/(j+2)! with 30 terms is used there.  Real or complex z.
    """
    z = _as_float(z)
    out = np.empty_like(z)
    small = np.abs(z) < 1.0
    zs = z[small]
    acc = np.zeros_like(zs)
    for j in range(29, -1, -1):
        acc = acc * zs + 1.0 / math.factorial(j + 2)
    out[small] = acc
    zb = z[~small]
    out[~small] = (np.expm1(zb) - zb) / (zb * zb)
    return out


# ---------------------------------------------------------------------------
# problem setup: symbols of A = exp(dt L), phi-weights, alpha-circulant data
# ---------------------------------------------------------------------------
@dataclass
class Setup:
    """Symbols and time tables of one Exp-ParaDiag instance.

    A = exp(dt L_h) acts per Fourier mode as E_k = exp(dt mu_k) (Sec. 2,
    eq. disc_wr).  Gamma_alpha = diag(alpha^{l/Nt}), lambda_{0,m} =
    alpha^{1/Nt} exp(2 pi i m/Nt) (Sec. 2, diagonalisation of C_0^alpha).
    """
    dim: int
    n: int
    Nt: int
    dt: float
    alpha: float
    a: float
    c: float = 0.0
    n1: float = 0.0
    n2: float = 0.0
    n3: float = 0.0
    scheme: int = 1
    b: tuple = (0.0, 0.0, 0.0)
    a_im: float = 0.0
    c_im: float = 0.0
    cstate: bool = False
    jac: int = 1            # IF1 preconditioner shift: see if1_sigma
    mu: np.ndarray = field(init=False, repr=False)
    E: np.ndarray = field(init=False, repr=False)
    w1: np.ndarray = field(init=False, repr=False)
    w2: np.ndarray = field(init=False, repr=False)
    gamma: np.ndarray = field(init=False, repr=False)
    lam: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        k = np.fft.fftfreq(self.n, 1.0 / self.n)
        grids = np.meshgrid(*([k] * self.dim), indexing="ij")
        k2 = sum(g * g for g in grids)
        self.mu = -self.a * k2 - self.c
        if self.a_im != 0.0 or self.c_im != 0.0:
            # complex coefficients (Schroedinger: a = i): complex state
            self.cstate = True
            self.mu = self.mu - 1j * (self.a_im * k2 + self.c_im)
        if any(bj != 0.0 for bj in self.b[:self.dim]):
            kd = k.copy()
            kd[self.n // 2] = 0.0        # first derivative of the Nyquist mode
            dgrids = np.meshgrid(*([kd] * self.dim), indexing="ij")
            self.mu = self.mu - 1j * sum(
                self.b[j] * dgrids[j] for j in range(self.dim))
        z = self.dt * self.mu
        self.E = np.exp(z)
        self.w1 = self.dt * phi1(z)
        self.w2 = self.dt * phi2(z)
        l = np.arange(self.Nt, dtype=np.float64)
        self.gamma = self.alpha ** (l / self.Nt)
        self.lam = self.alpha ** (1.0 / self.Nt) * np.exp(
            2j * np.pi * l / self.Nt)

    @classmethod
    def from_instance(cls, inst):
        return cls(inst.dim, inst.n, inst.Nt, inst.dt, inst.alpha, inst.a,
                   inst.c, inst.n1, inst.n2, inst.n3, inst.scheme,
                   tuple(getattr(inst, "b", (0.0, 0.0, 0.0))),
                   getattr(inst, "a_im", 0.0), getattr(inst, "c_im", 0.0),
                   bool(getattr(inst, "cstate", False)))

    @property
    def dtype(self):
        """Complex state (complex coefficients, or a complex u_0) or real."""
        return np.complex128 if self.cstate else np.float64

    def _out(self, w):
        return w if self.cstate else w.real

    @property
    def axes(self):
        """Spatial axes of a space-time array shaped (Nt, n, ..., n)."""
        return tuple(range(1, self.dim + 1))

    @property
    def nonlinear(self):
        return (self.n1, self.n2, self.n3) != (0.0, 0.0, 0.0)

    # -- functions of the spatial operator, applied through the spectrum --
    def spectral_apply(self, v, g):
        """g(L_h) v for one field v (shape (n,)*dim) or a stack (Nt, ...)."""
        axes = tuple(range(v.ndim - self.dim, v.ndim))
        return np.fft.ifftn(g * np.fft.fftn(v, axes=axes), axes=axes)

    def A(self, v):
        """A v with A = exp(dt L_h); real in, real out for a real state."""
        return self._out(self.spectral_apply(v, self.E))

    def W1(self, v):
        return self._out(self.spectral_apply(v, self.w1))

    def W2(self, v):
        return self._out(self.spectral_apply(v, self.w2))

    def N(self, u):
        return self.n1 * u + self.n2 * u * u + self.n3 * u * u * u

    def dN(self, u):
        return self.n1 + 2.0 * self.n2 * u + 3.0 * self.n3 * u * u


# ---------------------------------------------------------------------------
# O1: sequential time stepping (the plain definition of the result)
# ---------------------------------------------------------------------------
def sequential(st: Setup, u0):
    """u_1..u_Nt by sequential ETD1 / ETD2 stepping.

    Linear part: u_n = A u_{n-1} (Sec. 2, eq. disc_wr).  The all-at-once
    system Q u = f of Sec. 3 (eq. all_at_once_1storder) has exactly this
    block forward substitution as its solution.  Scheme EBDF2 steps by
    sequential_ebdf2.
    """
    if st.scheme == EBDF2:
        return sequential_ebdf2(st, u0)
    if ebdf_order(st.scheme):
        return sequential_ebdf(st, u0)
    if st.scheme == IF1:
        return sequential_if1(st, u0)
    U = np.empty((st.Nt,) + u0.shape, dtype=st.dtype)
    prev2, prev = u0, u0
    for j in range(st.Nt):
        un = st.A(prev)
        if st.nonlinear:
            if st.scheme == 1:
                un = un + st.W1(st.N(prev))
            else:
                un = un + st.W1(st.N(prev)) + st.W2(st.N(prev) - st.N(prev2))
        U[j] = un
        prev2, prev = prev, un
    return U


# ---------------------------------------------------------------------------
# all-at-once residual and the alpha-circulant preconditioner
# ---------------------------------------------------------------------------
def _shift(st, U, u_first):
    """(u_{n-1})_{n=1..Nt} with u_0 := u_first."""
    P = np.empty_like(U)
    P[0] = u_first
    P[1:] = U[:-1]
    return P


def nonlinear_term(st: Setup, u0, U):
    """G(U) + (nonlinear part of f): the slice-n term built from u_{n-1},
    u_{n-2} (u_{-1} := u_0), i.e. the lagged nonlinearity of Sec. 6.2."""
    if not st.nonlinear:
        return np.zeros_like(U)
    P1 = _shift(st, U, u0)
    N1 = st.N(P1)
    if st.scheme == 1:
        return st.W1(N1)
    P2 = _shift(st, P1, u0)
    N2 = st.N(P2)
    return st.W1(N1) + st.W2(N1 - N2)


def residual(st: Setup, u0, U):
    """R(U) = f + G(U) - Q U  (right-hand side of eq. pcond-1st-order).

    Q = I_t (x) I_x - C_0 (x) A, f = (A u_0 + [dt phi1 N(u_0)], 0, ..., 0).
    Slice n of R is A u_{n-1} + G_n - u_n with u_0 the initial condition.
    """
    P1 = _shift(st, U, u0)
    return st.A(P1) + nonlinear_term(st, u0, U) - U


def q_apply(st: Setup, V):
    """Q V with Q = I_t (x) I_x - C_0 (x) A (eq. all_at_once_1storder)."""
    return V - st.A(_shift(st, V, np.zeros_like(V[0])))


def qalpha_apply(st: Setup, V):
    """Q_alpha V with Q_alpha = I_t (x) I_x - C_0^alpha (x) A
    (eq. pcond-1st-order, C_0^alpha of eq. alpha_circ)."""
    P = _shift(st, V, st.alpha * V[-1])
    return V - st.A(P)


def time_dft(X):
    """(F (x) I_x) X with F = Nt^{-1/2} [omega^{(l1-1)(l2-1)}],
    omega = exp(+2 pi i/Nt) (Sec. 2)."""
    return np.fft.ifft(X, axis=0, norm="ortho")


def time_idft(X):
    """(F^* (x) I_x) X."""
    return np.fft.fft(X, axis=0, norm="ortho")


def precond_apply(st: Setup, R):
    """S = Q_alpha^{-1} R by the three steps of Sec. 3 (eq.
    exp_ParaDiag_steps):
      (a) S_a = (F (x) I)(Gamma_alpha (x) I) R
      (b) S_b,m = (I - lambda_{0,m} A)^{-1} S_a,m,  m = 1..Nt
      (c) S = (Gamma_alpha^{-1} (x) I)(F^* (x) I) S_b
    """
    g = st.gamma.reshape((st.Nt,) + (1,) * st.dim)
    Sa = time_dft(g * R)
    Sb = np.empty_like(Sa)
    for m in range(st.Nt):
        Sb[m] = st.spectral_apply(Sa[m], 1.0 / (1.0 - st.lam[m] * st.E))
    S = time_idft(Sb) / g
    return st._out(S)


def rel_err(U, V):
    """max_n ||u_n - v_n||_2 / max_n ||v_n||_2: the L_inf(0,T; L2) error
    of Sec. 6, normalised by the reference's norm."""
    ax = tuple(range(1, U.ndim))
    num = np.sqrt(np.sum(np.abs(U - V) ** 2, axis=ax)).max()
    den = np.sqrt(np.sum(np.abs(V) ** 2, axis=ax)).max()
    return num / den


# ---------------------------------------------------------------------------
# O2: the preconditioned fixed point (Richardson) iteration
# ---------------------------------------------------------------------------
def fixed_point(st: Setup, u0, U0=None, max_iter=200, tol=1e-11, ref=None,
                ref_tol=None, record=False):
    """u^{k+1} = u^k + s^k,  Q_alpha s^k = f + G(u^k) - Q u^k.

    Eq. pcond-1st-order (linear) with the nonlinearity lagged one iteration
    (Sec. 6.2); for EBDF2 the iteration of eq. pcond-2nd-order,
    v^{k+1} = v^k + R_alpha^{-1}(f_2 - R v^k), on slices 2..Nt, and its
    order-s analogue on slices s..Nt for EBDF3..EBDF6.
    U^0 = 0 unless given (Sec. 6 starts from zeros).
    Stops when ||s^k|| <= tol ||u^{k+1}||, or, if `ref` is given and
    ref_tol is set, when rel_err(u^{k+1}, ref) <= ref_tol.
    Returns (U, iterations, history) where history holds
    (||s||/||u||, rel_err vs ref or nan) per iteration and, if record,
    the iterates themselves.
    """
    U = np.zeros((st.Nt,) + u0.shape, dtype=st.dtype) if U0 is None \
        else U0.copy()
    hist, iterates = [], []
    bdf2 = st.scheme == EBDF2
    bdfs = ebdf_order(st.scheme) if not bdf2 else 0
    if1 = st.scheme == IF1
    for k in range(max_iter):
        if bdf2:
            R = residual_ebdf2(st, u0, U)
            S = precond_apply_ebdf2(st, R)
        elif bdfs:
            R = residual_ebdf(st, u0, U)
            S = precond_apply_ebdf(st, R)
        elif if1:
            R = residual_if1(st, u0, U)
            S = precond_apply_if1(st, R, if1_sigma(st, u0, U, k))
        else:
            R = residual(st, u0, U)
            S = precond_apply(st, R)
        U = U + S
        upd = np.linalg.norm(S) / max(np.linalg.norm(U), 1e-300)
        err = rel_err(U, ref) if ref is not None else float("nan")
        hist.append((upd, err))
        if record:
            iterates.append(U.copy())
        if ref is not None and ref_tol is not None:
            if err <= ref_tol:
                return U, k + 1, (hist, iterates)
        elif upd <= tol:
            return U, k + 1, (hist, iterates)
    return U, max_iter, (hist, iterates)


# ---------------------------------------------------------------------------
# O3: GMRES (left-preconditioned) and Newton-Krylov
# ---------------------------------------------------------------------------
def gmres(matvec, b, x0, restart=20, tol=1e-10, max_iter=200):
    """Restarted GMRES(m): Arnoldi with modified Gram-Schmidt and Givens
    rotations on the (m+1) x m Hessenberg matrix (Saad, Iterative Methods
    for Sparse Linear Systems, Alg. 6.9 with restarts).

    Stops when ||b - A x|| <= tol ||b||.  Returns (x, iterations, history of
    residual norms ||b - A x_k||, one per inner iteration, starting at k=0).
    """
    x = x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, [0.0]
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    hist = [beta]
    total = 0
    while total < max_iter and beta > tol * bnorm:
        m = restart
        V = np.zeros((m + 1, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r.ravel() / beta
        j_end = 0
        for j in range(m):
            w = matvec(V[j].reshape(b.shape)).ravel()
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= tol * bnorm or total >= max_iter:
                break
            nrm = np.linalg.norm(w)
            if nrm == 0.0:
                break
            V[j + 1] = w / nrm
        y = np.zeros(j_end)
        for i in range(j_end - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:j_end], y[i + 1:])) / H[i, i]
        x = x + (V[:j_end].T @ y).reshape(b.shape)
        r = b - matvec(x)
        beta = np.linalg.norm(r)
    return x, total, hist


def _real_view(st: Setup, op, b, x0):
    """A complex-state problem as a real one of twice the size (real and
    imaginary parts), on which the real GMRES runs with the inner product
    Re(x^H y)."""
    if not st.cstate:
        return op, b, x0, lambda x: x
    shape = b.shape
    to_r = lambda z: np.stack([z.real, z.imag])
    to_c = lambda r: r[0] + 1j * r[1]
    return (lambda r: to_r(op(to_c(r)))), to_r(b), to_r(x0), to_c


def gmres_solve(st: Setup, u0, restart=20, tol=1e-10, max_iter=200):
    """Linear problems: GMRES on Q_alpha^{-1} Q u = Q_alpha^{-1} f
    (Sec. 3.2, Theorem thm_gmres1 system), u^0 = 0."""
    zeros = np.zeros((st.Nt,) + u0.shape, dtype=st.dtype)
    f = residual(st, u0, zeros)          # f - Q*0
    b = precond_apply(st, f)
    op = lambda v: precond_apply(st, q_apply(st, v))
    rop, rb, rx0, back = _real_view(st, op, b, zeros)
    x, it, hist = gmres(rop, rb, rx0, restart, tol, max_iter)
    return back(x), it, hist


def gprime_apply(st: Setup, u0, U, V):
    """G'(U) V: derivative of the lagged nonlinear term with u_0 fixed."""
    if not st.nonlinear:
        return np.zeros_like(V)
    P1 = _shift(st, U, u0)
    V1 = _shift(st, V, np.zeros_like(u0))
    J1 = st.dN(P1) * V1
    if st.scheme == 1:
        return st.W1(J1)
    P2 = _shift(st, P1, u0)
    V2 = _shift(st, V1, np.zeros_like(u0))
    J2 = st.dN(P2) * V2
    return st.W1(J1) + st.W2(J1 - J2)


def newton_gmres(st: Setup, u0, restart=20, tol=1e-10, max_newton=30,
                 max_inner=200, eta_max=1e-3):
    """Newton on R(U) = 0 with inner GMRES(restart) on
    Q_alpha^{-1}(Q - G'(U)) d = Q_alpha^{-1} R(U), left-preconditioned by
    the Exp-ParaDiag step.  Forcing term eta_j = min(eta_max, ||R_j||/||R_0||).
    Stops when ||R_j|| <= tol ||R_0||.  Returns (U, newton_steps, inner_total,
    history of ||R_j||)."""
    U = np.zeros((st.Nt,) + u0.shape)
    R = residual(st, u0, U)
    r0 = np.linalg.norm(R)
    hist = [r0]
    inner_total = 0
    for j in range(max_newton):
        rn = np.linalg.norm(R)
        if rn <= tol * r0:
            return U, j, inner_total, hist
        eta = min(eta_max, rn / r0)
        Uc = U
        op = lambda v: precond_apply(st, q_apply(st, v)
                                     - gprime_apply(st, u0, Uc, v))
        b = precond_apply(st, R)
        d, it, _ = gmres(op, b, np.zeros_like(U), restart, eta, max_inner)
        inner_total += it
        U = U + d
        R = residual(st, u0, U)
        hist.append(np.linalg.norm(R))
    return U, max_newton, inner_total, hist


# ---------------------------------------------------------------------------
# O4: dense assembled operators for tiny sizes (brute force)
# ---------------------------------------------------------------------------
def _dft_matrix(n):
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def dense_operators(st: Setup):
    """Assemble A, Q, Q_alpha and the phi-weight matrices as dense real
    matrices from the definitions (Sec. 2 eq. st_system, Sec. 3 eq.
    all_at_once_1storder).  Only for n^dim * Nt up to a few thousand."""
    Fx = _dft_matrix(st.n)
    F = Fx
    for _ in range(st.dim - 1):
        F = np.kron(F, Fx)
    Finv = F.conj().T / F.shape[0]

    def dense_of(sym):
        M = Finv @ np.diag(sym.ravel()) @ F
        return M if st.cstate else M.real

    A = dense_of(st.E)
    Ns = A.shape[0]
    C0 = np.diag(np.ones(st.Nt - 1), -1)
    C0a = C0.copy()
    C0a[0, -1] = st.alpha
    I = np.eye(st.Nt * Ns)
    return {
        "A": A, "W1": dense_of(st.w1), "W2": dense_of(st.w2),
        "C0": C0, "C0a": C0a,
        "Q": I - np.kron(C0, A), "Qa": I - np.kron(C0a, A),
    }


def dense_solve(st: Setup, u0, D=None):
    """Linear all-at-once solve Q u = f by LU (numpy.linalg.solve)."""
    D = D or dense_operators(st)
    Ns = u0.size
    f = np.zeros(st.Nt * Ns, dtype=st.dtype)
    f[:Ns] = D["A"] @ u0.ravel()
    return np.linalg.solve(D["Q"], f).reshape((st.Nt,) + u0.shape)


def dense_newton(st: Setup, u0, tol=1e-14, max_iter=50, D=None):
    """Nonlinear all-at-once system R(U)=0 by dense Newton with LU."""
    D = D or dense_operators(st)
    Ns = u0.size
    Nt = st.Nt
    u0f = u0.ravel()
    U = np.zeros(Nt * Ns)

    def R_of(Uf):
        Us = Uf.reshape(Nt, Ns)
        P1 = np.vstack([u0f[None], Us[:-1]])
        P2 = np.vstack([u0f[None], P1[:-1]])
        out = (D["A"] @ P1.T).T - Us
        N1 = st.N(P1)
        if st.scheme == 1:
            out = out + (D["W1"] @ N1.T).T
        else:
            N2 = st.N(P2)
            out = out + (D["W1"] @ N1.T).T + (D["W2"] @ (N1 - N2).T).T
        return out.ravel()

    def J_of(Uf):
        Us = Uf.reshape(Nt, Ns)
        P1 = np.vstack([u0f[None], Us[:-1]])
        P2 = np.vstack([u0f[None], P1[:-1]])
        J = -np.eye(Nt * Ns) + np.kron(np.diag(np.ones(Nt - 1), -1), D["A"])
        for nn in range(1, Nt):
            d1 = st.dN(P1[nn])
            if st.scheme == 1:
                blk = D["W1"] * d1[None, :]
            else:
                blk = (D["W1"] + D["W2"]) * d1[None, :]
            J[nn * Ns:(nn + 1) * Ns, (nn - 1) * Ns:nn * Ns] += blk
            if st.scheme == 2 and nn >= 2:
                d2 = st.dN(P2[nn])
                J[nn * Ns:(nn + 1) * Ns, (nn - 2) * Ns:(nn - 1) * Ns] -= \
                    D["W2"] * d2[None, :]
        return J

    for _ in range(max_iter):
        R = R_of(U)
        if np.linalg.norm(R) <= tol * max(1.0, np.linalg.norm(U)):
            break
        U = U - np.linalg.solve(J_of(U), R)
    return U.reshape((Nt,) + u0.shape)


# ---------------------------------------------------------------------------
# EBDF2: the second-order exponential BDF of Sec. 4 (linear problems)
# ---------------------------------------------------------------------------
def ebdf2_tables(st: Setup):
    """Time tables of the (Nt-1)-slice system (Sec. 4, with Nt replaced by
    Nt-1 in the diagonalisation of Sec. 2): gamma_j = alpha^{j/(Nt-1)},
    lambda_{0,j} = alpha^{1/(Nt-1)} e^{2 pi i j/(Nt-1)} and, as the paper
    states them, lambda_{1,j} = alpha^{2/(Nt-1)} e^{4 pi i j/(Nt-1)},
    j = 0..Nt-2."""
    N = st.Nt - 1
    j = np.arange(N, dtype=np.float64)
    gamma = st.alpha ** (j / N)
    lam0 = st.alpha ** (1.0 / N) * np.exp(2j * np.pi * j / N)
    lam1 = st.alpha ** (2.0 / N) * np.exp(4j * np.pi * j / N)
    return gamma, lam0, lam1


def sequential_ebdf2(st: Setup, u0):
    """u_1..u_Nt of eq. 2nd_order_scheme: u_n = 4/3 A u_{n-1} - 1/3 B u_{n-2}
    with B = A^2, started from u_1 = A u_0."""
    U = np.empty((st.Nt,) + u0.shape, dtype=st.dtype)
    U[0] = st.A(u0)
    prev2, prev = u0, U[0]
    for j in range(1, st.Nt):
        U[j] = 4.0 / 3.0 * st.A(prev) - 1.0 / 3.0 * st.A(st.A(prev2))
        prev2, prev = prev, U[j]
    return U


def _B(st: Setup, v):
    """B v with B = A^2 (eq. 2nd_order_scheme), applied through the symbol."""
    return st._out(st.spectral_apply(v, st.E ** 2))


def r_apply_ebdf2(st: Setup, V):
    """R v for v = (v_2..v_Nt) with R = I - 4/3 C_0 (x) A + 1/3 C_1 (x) B
    (eq. all_at_once_2ndorder): row j is v_j - 4/3 A v_{j-1} + 1/3 B v_{j-2},
    entries before v_2 being zero."""
    out = V.copy()
    out[1:] -= 4.0 / 3.0 * st.A(V[:-1])
    out[2:] += 1.0 / 3.0 * _B(st, V[:-2])
    return out


def ralpha_apply_ebdf2(st: Setup, V):
    """R_alpha v with C_0^alpha, C_1^alpha of eq. pcond-2nd-order: C_1^alpha
    carries alpha at (1, Nt-2) and (2, Nt-1), C_0^alpha at (1, Nt-1)."""
    out = r_apply_ebdf2(st, V)
    a = st.alpha
    out[0] += -4.0 / 3.0 * a * st.A(V[-1]) + 1.0 / 3.0 * a * _B(st, V[-2])
    out[1] += 1.0 / 3.0 * a * _B(st, V[-1])
    return out


def residual_ebdf2(st: Setup, u0, U):
    """Residual of the EBDF2 window on slices u_1..u_Nt.

    Slice 1: A u_0 - u_1.  Slices 2..Nt: f_2 - R v (eq. all_at_once_2ndorder)
    with v = (u_2..u_Nt) and f_2 = (4/3 A u_1 - 1/3 B u_0, -1/3 B u_1, 0..)
    built from u_1 = A u_0, not from slice 1 of U.
    """
    u1 = st.A(u0)
    R = np.empty_like(U)
    R[0] = u1 - U[0]
    f2 = np.zeros_like(U[1:])
    f2[0] = 4.0 / 3.0 * st.A(u1) - 1.0 / 3.0 * _B(st, u0)
    if st.Nt > 2:
        f2[1] = -1.0 / 3.0 * _B(st, u1)
    R[1:] = f2 - r_apply_ebdf2(st, U[1:])
    return R


def precond_apply_ebdf2(st: Setup, R):
    """Slice 1 unchanged; slices 2..Nt: R_alpha^{-1} by the three steps of
    eq. exp_ParaDiag_steps_2ndorder with Nt-1 time points:
      (a) S_p = (F (x) I)(Gamma_alpha (x) I) r
      (b) S_q,j = (I - 4/3 lambda_{0,j} A + 1/3 lambda_{1,j} B)^{-1} S_p,j
      (c) s = (Gamma_alpha^{-1} (x) I)(F^* (x) I) S_q
    """
    gamma, lam0, lam1 = ebdf2_tables(st)
    N = st.Nt - 1
    g = gamma.reshape((N,) + (1,) * st.dim)
    Sp = time_dft(g * R[1:])
    Sq = np.empty_like(Sp)
    E = st.E
    for j in range(N):
        sym = 1.0 - 4.0 / 3.0 * lam0[j] * E + 1.0 / 3.0 * lam1[j] * E * E
        Sq[j] = st.spectral_apply(Sp[j], 1.0 / sym)
    S = np.empty_like(R)
    S[0] = R[0]
    S[1:] = st._out(time_idft(Sq) / g)
    return S


def gmres_solve_ebdf2(st: Setup, u0, restart=20, tol=1e-10, max_iter=200):
    """GMRES on R_alpha^{-1} R v = R_alpha^{-1} f_2 (Sec. 4.2), v^0 = 0;
    returns the window u_1..u_Nt with u_1 = A u_0."""
    zeros = np.zeros((st.Nt,) + u0.shape, dtype=st.dtype)
    f2 = residual_ebdf2(st, u0, zeros)[1:]

    def prec(v):
        full = np.zeros((st.Nt,) + u0.shape, dtype=st.dtype)
        full[1:] = v
        return precond_apply_ebdf2(st, full)[1:]

    b = prec(f2)
    op = lambda v: prec(r_apply_ebdf2(st, v))
    rop, rb, rx0, back = _real_view(st, op, b, np.zeros_like(f2))
    v, it, hist = gmres(rop, rb, rx0, restart, tol, max_iter)
    v = back(v)
    U = np.empty((st.Nt,) + u0.shape, dtype=st.dtype)
    U[0] = st.A(u0)
    U[1:] = v
    return U, it, hist


def dense_operators_ebdf2(st: Setup):
    """Dense A, B, C_0, C_1, their alpha-circulant versions, R, R_alpha
    (eqs. all_at_once_2ndorder, alpha_circ_c1, pcond-2nd-order), assembled
    entry by entry for (Nt-1) time slices."""
    D = dense_operators(st)
    A = D["A"]
    B = A @ A
    N = st.Nt - 1
    C0 = np.diag(np.ones(N - 1), -1)
    C1 = np.diag(np.ones(N - 2), -2)
    C0a = C0.copy()
    C0a[0, N - 1] = st.alpha
    C1a = C1.copy()
    C1a[0, N - 2] = st.alpha
    C1a[1, N - 1] = st.alpha
    I = np.eye(N * A.shape[0])
    return {
        "A": A, "B": B, "C0": C0, "C1": C1, "C0a": C0a, "C1a": C1a,
        "R": I - 4.0 / 3.0 * np.kron(C0, A) + 1.0 / 3.0 * np.kron(C1, B),
        "Ra": I - 4.0 / 3.0 * np.kron(C0a, A) + 1.0 / 3.0 * np.kron(C1a, B),
    }


# ---------------------------------------------------------------------------
# IF1: the implicit integrating-factor scheme of Sec. 5
# ---------------------------------------------------------------------------
def sequential_if1(st: Setup, u0, tol=1e-15, max_newton=60):
    """u_1..u_Nt of eq. fully_discrete_nonlinear,
    u_n = A u_{n-1} + dt N(u_n): N acts pointwise, so each step is one
    scalar equation u - dt N(u) = (A u_{n-1})(x) per grid point, solved by
    Newton's method from u = (A u_{n-1})(x) to round-off."""
    U = np.empty((st.Nt,) + u0.shape, dtype=st.dtype)
    prev = u0
    for n in range(st.Nt):
        rhs = st.A(prev)
        u = rhs.copy()
        for _ in range(max_newton):
            du = (u - st.dt * st.N(u) - rhs) / (1.0 - st.dt * st.dN(u))
            u = u - du
            if np.max(np.abs(du)) <= tol * max(1.0, np.max(np.abs(u))):
                break
        U[n] = u
        prev = u
    return U


def residual_if1(st: Setup, u0, U):
    """R(U) = f + dt N_0(U) - Q U (the all-at-once form of eq.
    fully_discrete_nonlinear): slice n is A u_{n-1} + dt N(u_n) - u_n."""
    P1 = _shift(st, U, u0)
    return st.A(P1) + st.dt * st.N(U) - U


def if1_sigma(st: Setup, u0, U, k):
    """Scalar Jacobian shift of the IF1 preconditioner Q_alpha - sigma I.
    jac = 0: sigma = 0, the lagged iteration of eq. disc_imextype_scheme;
    jac = 1: dt times the space-time mean of N'(U^k) (the averaged Jacobian
    of eq. newton_2, averaged over space as well), from u_0 at the first
    iteration; jac = 2: dt times the spatial mean of N'(u_0) (the
    Jacobian-at-u_0 variant of Sec. 5, averaged over space)."""
    if st.jac == 0:
        return 0.0
    if st.jac == 2 or k == 0:
        return st.dt * float(np.mean(st.dN(u0)).real)
    return st.dt * float(np.mean(st.dN(U)).real)


def precond_apply_if1(st: Setup, R, sigma):
    """(Q_alpha - sigma I)^{-1} R by the steps of eq.
    exp_ParaDiag_steps_newton with the averaged Jacobian reduced to the
    scalar sigma = dt nbar, so that step (b) stays pointwise:
    S_q,m = (I - lambda_{0,m} A - sigma)^{-1} S_p,m."""
    g = st.gamma.reshape((st.Nt,) + (1,) * st.dim)
    Sa = time_dft(g * R)
    Sb = np.empty_like(Sa)
    for m in range(st.Nt):
        Sb[m] = st.spectral_apply(Sa[m], 1.0 / (1.0 - st.lam[m] * st.E - sigma))
    return st._out(time_idft(Sb) / g)


def dense_newton_if1(st: Setup, u0, tol=1e-14, max_iter=50, D=None):
    """The all-at-once IF1 system (I - C_0 (x) A) U - dt N_0(U) = f by dense
    Newton with LU on the assembled Jacobian."""
    D = D or dense_operators(st)
    Ns, Nt = u0.size, st.Nt
    f = np.zeros(Nt * Ns)
    f[:Ns] = D["A"] @ u0.ravel()
    U = np.zeros(Nt * Ns)
    for _ in range(max_iter):
        R = D["Q"] @ U - st.dt * st.N(U) - f
        if np.linalg.norm(R) <= tol * max(1.0, np.linalg.norm(U)):
            break
        J = D["Q"] - st.dt * np.diag(st.dN(U))
        U = U - np.linalg.solve(J, R)
    return U.reshape((Nt,) + u0.shape)


def outer_iteration_if1(st: Setup, u0, iters, D=None):
    """The paper's Exp-ParaDiag iteration for IF1 (eq. fully_disc_wr_nonlinear)
    with exact inner solves: U^k solves (I - C_0^alpha (x) A) U - dt N_0(U)
    = b^{k-1}, b^{k-1} = (A (u_0 - alpha u_Nt^{k-1}), 0, .., 0), by dense
    Newton; U^0 = 0.  Returns the iterates."""
    D = D or dense_operators(st)
    Ns, Nt = u0.size, st.Nt
    U = np.zeros(Nt * Ns)
    out = []
    for _ in range(iters):
        b = np.zeros(Nt * Ns)
        b[:Ns] = D["A"] @ (u0.ravel() - st.alpha * U[-Ns:])
        V = U.copy()
        for _ in range(50):
            R = D["Qa"] @ V - st.dt * st.N(V) - b
            if np.linalg.norm(R) <= 1e-15 * max(1.0, np.linalg.norm(V)):
                break
            V = V - np.linalg.solve(D["Qa"] - st.dt * np.diag(st.dN(V)), R)
        U = V
        out.append(U.reshape((Nt,) + u0.shape).copy())
    return out


# ---------------------------------------------------------------------------
# EBDF3..EBDF6: the exponential BDF schemes of order s of Sec. bdfs
# ---------------------------------------------------------------------------
# u_n = sum_{j=1..s} beta_j A^j u_{n-j}, n >= s, with the coefficients the
# paper prints in eqs. 3rd_order_scheme, fourth_order_scheme,
# fifth_order_scheme and sixth_order_scheme (order 2: eq. 2nd_order_scheme),
# as (numerator, denominator) pairs.
EBDF_COEFFS = {
    2: ((4, -1), 3),
    3: ((18, -9, 2), 11),
    4: ((48, -36, 16, -3), 25),
    5: ((300, -300, 200, -75, 12), 137),
    6: ((360, -450, 400, -225, 72, -10), 147),
}


def ebdf_order(scheme):
    """Order s of an exponential BDF scheme code (EBDF2 = 3, EBDF3..EBDF6 =
    5..8), 0 for the other schemes."""
    if scheme == EBDF2:
        return 2
    return scheme - 2 if scheme in (EBDF3, EBDF4, EBDF5, EBDF6) else 0


def ebdf_beta(s):
    """beta_1..beta_s of the order-s scheme as floats."""
    num, den = EBDF_COEFFS[s]
    return [b / den for b in num]


def _Apow(st: Setup, v, j):
    """A^j v through the symbol E^j (j >= 0)."""
    if j == 0:
        return v.copy()
    return st._out(st.spectral_apply(v, st.E ** j))


def ebdf_tables(st: Setup, s):
    """Time tables of the N = Nt - s + 1 slice system: gamma_l =
    alpha^{l/N}, lambda_{0,m} = alpha^{1/N} e^{2 pi i m/N} and the
    eigenvalues lambda_{0,m}^j of C_{j-1}^alpha, j = 1..s (reading:
    C_{j-1}^alpha = (C_0^alpha)^j, which is what the alpha positions the
    paper gives for C_1..C_5 describe)."""
    N = st.Nt - s + 1
    l = np.arange(N, dtype=np.float64)
    gamma = st.alpha ** (l / N)
    lam0 = st.alpha ** (1.0 / N) * np.exp(2j * np.pi * l / N)
    lams = [lam0 ** j for j in range(1, s + 1)]
    return gamma, lams


def _ebdf_start(st: Setup, u0, s):
    """Slices u_0..u_{s-1}: u_0 and the start values u_j = A^j u_0 (the
    exact exponential steps; the paper leaves u_1..u_{s-1} open)."""
    return [u0] + [_Apow(st, u0, j) for j in range(1, s)]


def sequential_ebdf(st: Setup, u0, s=None):
    """u_1..u_Nt of the order-s exponential BDF, started from u_j = A^j u_0,
    j < s."""
    s = s or ebdf_order(st.scheme)
    beta = ebdf_beta(s)
    hist = _ebdf_start(st, u0, s)
    for n in range(s, st.Nt + 1):
        un = sum(beta[j - 1] * _Apow(st, hist[n - j], j)
                 for j in range(1, s + 1))
        hist.append(un)
    return np.array(hist[1:st.Nt + 1], dtype=st.dtype)


def r_apply_ebdf(st: Setup, V, s=None):
    """R_s v, R_s = I - sum_j beta_j C_{j-1} (x) A^j (eqs.
    all_at_once_3rdorder .. all_at_once_6thorder), v = (v_s..v_Nt): row i
    is v_i - sum_j beta_j A^j v_{i-j}, entries before v_s being zero."""
    s = s or ebdf_order(st.scheme)
    beta = ebdf_beta(s)
    out = V.copy()
    for j in range(1, s + 1):
        if j < V.shape[0]:
            out[j:] -= beta[j - 1] * _Apow(st, V[:-j], j)
    return out


def ralpha_apply_ebdf(st: Setup, V, s=None):
    """R_s^alpha v: C_{j-1}^alpha adds alpha at rows i = 0..j-1, columns
    N - j + i (0-based), the positions the paper lists."""
    s = s or ebdf_order(st.scheme)
    beta = ebdf_beta(s)
    N = V.shape[0]
    out = r_apply_ebdf(st, V, s)
    for j in range(1, s + 1):
        for i in range(min(j, N)):
            out[i] -= beta[j - 1] * st.alpha * _Apow(st, V[N - j + i], j)
    return out


def residual_ebdf(st: Setup, u0, U, s=None):
    """Residual of the order-s window on slices u_1..u_Nt.

    Start slices j = 1..s-1: A^j u_0 - u_j.  Slices n = s..Nt: f_s - R_s v
    with v = (u_s..u_Nt), f_s built from u_0 and the start values A^j u_0
    (not from U's start slices), i.e. sum_j beta_j A^j w_{n-j} - u_n with
    w_m = u_m for m >= s and A^m u_0 below.
    """
    s = s or ebdf_order(st.scheme)
    beta = ebdf_beta(s)
    start = _ebdf_start(st, u0, s)
    R = np.empty_like(U)
    for j in range(1, s):
        R[j - 1] = start[j] - U[j - 1]
    for n in range(s, st.Nt + 1):
        acc = np.zeros_like(U[0])
        for j in range(1, s + 1):
            m = n - j
            w = U[m - 1] if m >= s else start[m]
            acc = acc + beta[j - 1] * _Apow(st, w, j)
        R[n - 1] = acc - U[n - 1]
    return R


def precond_apply_ebdf(st: Setup, R, s=None):
    """Start slices unchanged; slices s..Nt: (R_s^alpha)^{-1} by steps
    (a)-(c) on N = Nt - s + 1 time points, step (b) inverting
    I - sum_j beta_j lambda_{j-1,m} A^j per frequency m."""
    s = s or ebdf_order(st.scheme)
    beta = ebdf_beta(s)
    gamma, lams = ebdf_tables(st, s)
    N = st.Nt - s + 1
    o = s - 1
    g = gamma.reshape((N,) + (1,) * st.dim)
    Sp = time_dft(g * R[o:])
    Sq = np.empty_like(Sp)
    for m in range(N):
        sym = 1.0 - sum(beta[j - 1] * lams[j - 1][m] * st.E ** j
                        for j in range(1, s + 1))
        Sq[m] = st.spectral_apply(Sp[m], 1.0 / sym)
    S = np.empty_like(R)
    S[:o] = R[:o]
    S[o:] = st._out(time_idft(Sq) / g)
    return S


def gmres_solve_ebdf(st: Setup, u0, restart=20, tol=1e-10, max_iter=200,
                     s=None):
    """GMRES on (R_s^alpha)^{-1} R_s v = (R_s^alpha)^{-1} f_s, v^0 = 0
    (the GMRES preconditioners of Sec. bdfs); returns the window with the
    start slices A^j u_0."""
    s = s or ebdf_order(st.scheme)
    o = s - 1
    zeros = np.zeros((st.Nt,) + u0.shape, dtype=st.dtype)
    fs = residual_ebdf(st, u0, zeros, s)[o:]

    def prec(v):
        full = np.zeros((st.Nt,) + u0.shape, dtype=st.dtype)
        full[o:] = v
        return precond_apply_ebdf(st, full, s)[o:]

    b = prec(fs)
    op = lambda v: prec(r_apply_ebdf(st, v, s))
    rop, rb, rx0, back = _real_view(st, op, b, np.zeros_like(fs))
    v, it, hist = gmres(rop, rb, rx0, restart, tol, max_iter)
    U = np.empty((st.Nt,) + u0.shape, dtype=st.dtype)
    U[:o] = np.array(_ebdf_start(st, u0, s)[1:], dtype=st.dtype).reshape(
        (o,) + u0.shape)
    U[o:] = back(v)
    return U, it, hist


def dense_operators_ebdf(st: Setup, s=None):
    """Dense A, A^j, C_{j-1}, C_{j-1}^alpha (alpha entries placed at the
    positions the paper lists for C_1..C_5), R_s and R_s^alpha for
    N = Nt - s + 1 slices, assembled entry by entry."""
    s = s or ebdf_order(st.scheme)
    beta = ebdf_beta(s)
    D = dense_operators(st)
    A = D["A"]
    N = st.Nt - s + 1
    Ap = [np.eye(A.shape[0])]
    for _ in range(s):
        Ap.append(Ap[-1] @ A)
    C, Ca = [], []
    for j in range(1, s + 1):
        Cj = np.zeros((N, N))
        for i in range(j, N):
            Cj[i, i - j] = 1.0
        Cja = Cj.copy()
        for i in range(min(j, N)):
            Cja[i, N - j + i] = st.alpha
        C.append(Cj)
        Ca.append(Cja)
    I = np.eye(N * A.shape[0])
    R = I - sum(beta[j - 1] * np.kron(C[j - 1], Ap[j]) for j in range(1, s + 1))
    Ra = I - sum(beta[j - 1] * np.kron(Ca[j - 1], Ap[j])
                 for j in range(1, s + 1))
    return {"A": A, "Ap": Ap, "C": C, "Ca": Ca, "R": R, "Ra": Ra}


# ---------------------------------------------------------------------------
# BiCGStab with the Exp-ParaDiag preconditioner (the bracketed timings of
# Table cpu_time_combined)
# ---------------------------------------------------------------------------
def bicgstab(matvec, b, x0, tol=1e-10, max_iter=200):
    """BiCGStab (van der Vorst 1992; Saad, Iterative Methods for Sparse
    Linear Systems, Alg. 7.7) on matvec(x) = b with shadow vector r^_0 =
    r_0.  Stops when ||r_j|| <= tol ||b|| (r_j the recurred residual) or
    when an intermediate s_j is that small.  Returns (x, iterations,
    history of ||r_j||)."""
    x = x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, [0.0]
    r = b - matvec(x)
    rhat = r.copy()
    hist = [np.linalg.norm(r)]
    if hist[0] <= tol * bnorm:
        return x, 0, hist
    p = r.copy()
    rho = np.vdot(rhat, r).real
    it = 0
    while it < max_iter:
        v = matvec(p)
        al = rho / np.vdot(rhat, v).real
        s = r - al * v
        it += 1
        sn = np.linalg.norm(s)
        if sn <= tol * bnorm:
            x = x + al * p
            hist.append(sn)
            break
        t = matvec(s)
        om = np.vdot(t, s).real / np.vdot(t, t).real
        x = x + al * p + om * s
        r = s - om * t
        hist.append(np.linalg.norm(r))
        if hist[-1] <= tol * bnorm:
            break
        rho_new = np.vdot(rhat, r).real
        be = (rho_new / rho) * (al / om)
        rho = rho_new
        p = r + be * (p - om * v)
    return x, it, hist


def bicgstab_solve(st: Setup, u0, tol=1e-10, max_iter=200):
    """Linear problems: BiCGStab on the left-preconditioned system GMRES
    solves (Q_alpha^{-1} Q u = Q_alpha^{-1} f; for the exponential BDF
    schemes (R^alpha)^{-1} R v = (R^alpha)^{-1} f on the unknown slices),
    u^0 = 0.  Returns (U, iterations, history)."""
    s = ebdf_order(st.scheme)
    if s:
        o = s - 1
        zeros = np.zeros((st.Nt,) + u0.shape, dtype=st.dtype)
        fs = residual_ebdf(st, u0, zeros, s)[o:]

        def prec(v):
            full = np.zeros((st.Nt,) + u0.shape, dtype=st.dtype)
            full[o:] = v
            return precond_apply_ebdf(st, full, s)[o:]

        b = prec(fs)
        op = lambda v: prec(r_apply_ebdf(st, v, s))
        rop, rb, rx0, back = _real_view(st, op, b, np.zeros_like(fs))
        v, it, hist = bicgstab(rop, rb, rx0, tol, max_iter)
        U = np.empty((st.Nt,) + u0.shape, dtype=st.dtype)
        U[:o] = np.array(_ebdf_start(st, u0, s)[1:], dtype=st.dtype).reshape(
            (o,) + u0.shape)
        U[o:] = back(v)
        return U, it, hist
    zeros = np.zeros((st.Nt,) + u0.shape, dtype=st.dtype)
    b = precond_apply(st, residual(st, u0, zeros))
    op = lambda v: precond_apply(st, q_apply(st, v))
    rop, rb, rx0, back = _real_view(st, op, b, zeros)
    x, it, hist = bicgstab(rop, rb, rx0, tol, max_iter)
    return back(x), it, hist


def newton_bicgstab(st: Setup, u0, tol=1e-10, max_newton=30, max_inner=200,
                    eta_max=1e-3):
    """newton_gmres with BiCGStab as the inner solver of
    Q_alpha^{-1}(Q - G'(U)) d = Q_alpha^{-1} R(U) (ETD1/ETD2 with the
    lagged nonlinearity).  Returns (U, newton_steps, inner_total, history of
    ||R_j||)."""
    U = np.zeros((st.Nt,) + u0.shape)
    R = residual(st, u0, U)
    r0 = np.linalg.norm(R)
    hist = [r0]
    inner_total = 0
    for j in range(max_newton):
        rn = np.linalg.norm(R)
        if rn <= tol * r0:
            return U, j, inner_total, hist
        eta = min(eta_max, rn / r0)
        Uc = U
        op = lambda v: precond_apply(st, q_apply(st, v)
                                     - gprime_apply(st, u0, Uc, v))
        d, it, _ = bicgstab(op, precond_apply(st, R), np.zeros_like(U), eta,
                            max_inner)
        inner_total += it
        U = U + d
        R = residual(st, u0, U)
        hist.append(np.linalg.norm(R))
    return U, max_newton, inner_total, hist
