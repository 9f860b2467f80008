"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here retypes the oracle's own formulas: each check compares the
oracle with something independent of it (mpmath at 50 digits, the explicit
DFT matrices of the definitions, dense LU on the assembled all-at-once
matrices, closed forms derived from the paper's iteration matrix, the
textbook convergence order, scipy's GMRES).
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg

import oracle as O
import workloads as W

mpmath.mp.dps = 50


def _field(rng, dim, n):
    return rng.uniform(-0.9, 0.9, size=(n,) * dim)


# ---------------------------------------------------------------------------
# phi functions: mpmath, 50 digits
# ---------------------------------------------------------------------------
def _mp_phi1(z):
    z = mpmath.mpf(z)
    return mpmath.mpf(1) if z == 0 else mpmath.expm1(z) / z


def _mp_phi2(z):
    z = mpmath.mpf(z)
    return mpmath.mpf(1) / 2 if z == 0 else (mpmath.expm1(z) - z) / (z * z)


ZS = np.concatenate([-np.logspace(-12, 4, 60), np.logspace(-12, 0.5, 20),
                     [0.0, -0.1, 0.1, -1.0, 1.0, -0.999999, 0.999999]])


def test_phi1_phi2_vs_mpmath():
    p1 = O.phi1(ZS)
    p2 = O.phi2(ZS)
    for z, a, b in zip(ZS, p1, p2):
        r1 = float(_mp_phi1(float(z)))
        r2 = float(_mp_phi2(float(z)))
        assert abs(a - r1) <= 4.5e-16 * abs(r1), (z, a, r1)
        assert abs(b - r2) <= 9e-16 * abs(r2), (z, b, r2)


# ---------------------------------------------------------------------------
# spatial operator: symbol and exp(dt L) from independent constructions
# ---------------------------------------------------------------------------
def test_symbol_is_laplacian_on_trig_polynomials():
    st = O.Setup(2, 16, 4, 0.1, 1e-2, a=0.3, c=0.2)
    x = 2 * np.pi * np.arange(16) / 16
    X, Y = np.meshgrid(x, x, indexing="ij")
    v = np.sin(3 * X) * np.cos(2 * Y) + np.cos(8 * Y)   # includes Nyquist
    Lv = st.spectral_apply(v, st.mu).real
    # a * Lap(v) - c v, analytically
    exact = (-0.3 * 13 - 0.2) * np.sin(3 * X) * np.cos(2 * Y) \
        + (-0.3 * 64 - 0.2) * np.cos(8 * Y)
    assert np.max(np.abs(Lv - exact)) < 1e-12


def test_A_is_matrix_exponential_of_dense_L():
    st = O.Setup(1, 12, 4, 0.07, 1e-2, a=0.5, c=0.1)
    j = np.arange(12)
    F = np.exp(-2j * np.pi * np.outer(j, j) / 12)
    L = (F.conj().T / 12 @ np.diag(st.mu) @ F).real
    A = scipy.linalg.expm(st.dt * L)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(12)
    assert np.max(np.abs(A @ v - st.A(v))) < 1e-13
    D = O.dense_operators(st)
    assert np.max(np.abs(D["A"] - A)) < 1e-13


# ---------------------------------------------------------------------------
# time DFT F and the diagonalisation of C_0^alpha (Sec. 2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("Nt", [2, 5, 8, 16])
def test_time_dft_is_papers_F(Nt):
    omega = np.exp(2j * np.pi / Nt)
    l = np.arange(Nt)
    F = omega ** np.outer(l, l) / np.sqrt(Nt)
    rng = np.random.default_rng(Nt)
    X = rng.standard_normal((Nt, 3)) + 1j * rng.standard_normal((Nt, 3))
    assert np.allclose(O.time_dft(X), F @ X, atol=1e-14)
    assert np.allclose(O.time_idft(X), F.conj().T @ X, atol=1e-14)


@pytest.mark.parametrize("Nt,alpha", [(4, 0.3), (8, 1e-2), (16, 1e-3)])
def test_alpha_circulant_diagonalisation(Nt, alpha):
    st = O.Setup(1, 4, Nt, 0.1, alpha, a=1.0)
    omega = np.exp(2j * np.pi / Nt)
    l = np.arange(Nt)
    F = omega ** np.outer(l, l) / np.sqrt(Nt)
    G = np.diag(st.gamma)
    P = np.linalg.inv(G) @ F.conj().T
    C0a = np.diag(np.ones(Nt - 1), -1)
    C0a[0, -1] = alpha
    rebuilt = P @ np.diag(st.lam) @ np.linalg.inv(P)
    assert np.max(np.abs(rebuilt - C0a)) < 1e-12


# ---------------------------------------------------------------------------
# Pi2: single Fourier mode of the heat equation (ETD1 exact in time)
# ---------------------------------------------------------------------------
def test_single_mode_heat_exact():
    n, Nt, T = 16, 8, 1.0
    st = O.Setup(1, n, Nt, T / Nt, 1e-2, a=1.0)
    x = 2 * np.pi * np.arange(n) / n
    u0 = np.sin(x)
    U = O.sequential(st, u0)
    exact = np.array([np.exp(-(k + 1) * T / Nt) * np.sin(x)
                      for k in range(Nt)])
    assert np.max(np.abs(U - exact)) < 1e-15
    Ufp, it, _ = O.fixed_point(st, u0, tol=1e-15, max_iter=20)
    assert np.max(np.abs(Ufp - exact)) < 1e-15


# ---------------------------------------------------------------------------
# Pi1: closed form of every linear iterate (from eq. pcond_system)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n,Nt,alpha,a,c", [
    (1, 16, 8, 1e-2, 1.0, 0.0),
    (1, 64, 16, 1e-2, 1.0, 0.0),
    (2, 8, 8, 0.2, 0.05, 0.3),
    (2, 8, 4, 1e-3, 0.01, 0.0),
])
def test_linear_iterates_closed_form(dim, n, Nt, alpha, a, c):
    st = O.Setup(dim, n, Nt, 1.0 / Nt, alpha, a=a, c=c)
    rng = np.random.default_rng(7)
    u0 = _field(rng, dim, n)
    _, _, (hist, its) = O.fixed_point(st, u0, max_iter=4, tol=0.0,
                                      record=True)
    axes = tuple(range(dim))
    u0h = np.fft.fftn(u0, axes=axes)
    ET = st.E ** Nt
    psi = -alpha * ET / (1.0 - alpha * ET)
    for k, Uk in enumerate(its, start=1):
        for m in range(Nt):
            pred = (1.0 - psi ** k) * st.E ** (m + 1) * u0h
            got = np.fft.fftn(Uk[m], axes=axes)
            assert np.max(np.abs(got - pred)) <= 1e-13 * np.max(np.abs(u0h))


def test_heat1d_workload_iteration_count_from_contraction():
    """The 1D heat workload: |psi_1| = alpha e^{-T}/(1 - alpha e^{-T}); the
    iteration count to 1e-10 (relative L_inf(L2) error) is the smallest k
    with max over present modes |psi|^k below the tolerance."""
    inst = W.heat1d()
    st = O.Setup.from_instance(inst)
    ref = O.sequential(st, inst.u0)
    _, it, _ = O.fixed_point(st, inst.u0, ref=ref, ref_tol=1e-10,
                             max_iter=50)
    psi1 = inst.alpha * math.exp(-inst.T) / (1 - inst.alpha * math.exp(-inst.T))
    assert abs(psi1 - 3.69e-3) < 1e-5
    # slowest present mode is |k|=1 (no mean mode in u0)
    k_pred = math.ceil(math.log(1e-10) / math.log(psi1))
    assert it in (k_pred - 1, k_pred)


def test_contraction_bound_thm_1st():
    """Theorem thm_1st: error contraction per iteration is at most
    alpha e^{lam_max T}/(1 - alpha e^{lam_max T})."""
    st = O.Setup(1, 32, 16, 1.0 / 16, 0.05, a=0.2, c=0.05)
    rng = np.random.default_rng(3)
    u0 = _field(rng, 1, 32)
    ref = O.sequential(st, u0)
    _, _, (hist, its) = O.fixed_point(st, u0, max_iter=5, tol=0.0,
                                      record=True)
    lam_max = -st.c
    bound = st.alpha * math.exp(lam_max * 1.0) / (
        1 - st.alpha * math.exp(lam_max * 1.0))
    errs = [np.sqrt(((ref) ** 2).sum(axis=1)).max()] + [
        np.sqrt(((U - ref) ** 2).sum(axis=1)).max() for U in its]
    for k in range(1, len(errs)):
        assert errs[k] <= bound ** k * errs[0] * (1 + 1e-9) + 1e-15


# ---------------------------------------------------------------------------
# Pi3: dense assembled matrices solved by LU
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n,Nt", [(1, 8, 6), (1, 12, 8), (2, 4, 4)])
def test_sequential_equals_dense_lu(dim, n, Nt):
    st = O.Setup(dim, n, Nt, 0.1, 1e-2, a=0.7, c=0.05)
    u0 = _field(np.random.default_rng(11), dim, n)
    Ud = O.dense_solve(st, u0)
    assert O.rel_err(O.sequential(st, u0), Ud) < 1e-14


@pytest.mark.parametrize("dim,n,Nt,alpha", [(1, 12, 8, 1e-2), (2, 4, 4, 0.3),
                                            (1, 8, 6, 1e-3)])
def test_precond_apply_equals_dense_inverse(dim, n, Nt, alpha):
    st = O.Setup(dim, n, Nt, 0.1, alpha, a=0.4)
    D = O.dense_operators(st)
    rng = np.random.default_rng(5)
    R = rng.standard_normal((Nt,) + (n,) * dim)
    S = O.precond_apply(st, R)
    Sd = np.linalg.solve(D["Qa"], R.ravel()).reshape(R.shape)
    assert np.max(np.abs(S - Sd)) < 1e-12 * np.max(np.abs(Sd)) / alpha ** 0
    # and the operator applications agree with the dense matrices
    assert np.allclose(O.q_apply(st, R).ravel(), D["Q"] @ R.ravel(),
                       atol=1e-13)
    assert np.allclose(O.qalpha_apply(st, R).ravel(), D["Qa"] @ R.ravel(),
                       atol=1e-13)


def test_residual_equals_dense_f_minus_QU():
    st = O.Setup(1, 8, 5, 0.1, 1e-2, a=0.9)
    D = O.dense_operators(st)
    rng = np.random.default_rng(2)
    u0 = _field(rng, 1, 8)
    U = rng.standard_normal((5, 8))
    f = np.zeros(40)
    f[:8] = D["A"] @ u0
    R = O.residual(st, u0, U)
    assert np.allclose(R.ravel(), f - D["Q"] @ U.ravel(), atol=1e-14)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("dim,n,Nt", [(1, 8, 6), (2, 4, 4)])
def test_nonlinear_sequential_equals_dense_newton(scheme, dim, n, Nt):
    st = O.Setup(dim, n, Nt, 0.05, 1e-2, a=0.3, n1=1.0, n2=-0.4, n3=-1.0,
                 scheme=scheme)
    u0 = _field(np.random.default_rng(4), dim, n)
    Ud = O.dense_newton(st, u0)
    assert O.rel_err(O.sequential(st, u0), Ud) < 1e-13


# ---------------------------------------------------------------------------
# Pi4: spectrum of Q_alpha^{-1} Q (Lemma gmres_centered_at1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("c", [0.0, 0.2])
def test_preconditioned_spectrum(c):
    st = O.Setup(1, 8, 5, 0.1, 0.05, a=0.6, c=c)
    D = O.dense_operators(st)
    ev = np.linalg.eigvals(np.linalg.solve(D["Qa"], D["Q"]))
    ET = st.E ** st.Nt
    pred = np.concatenate([np.ones(8 * 4), 1.0 / (1.0 - st.alpha * ET)])
    assert np.allclose(np.sort_complex(ev), np.sort_complex(pred + 0j),
                       atol=1e-10)
    radius = np.max(np.abs(ev - 1))
    assert radius <= st.alpha / (1 - st.alpha) + 1e-12
    if c == 0.0:
        assert abs(radius - st.alpha / (1 - st.alpha)) < 1e-12


# ---------------------------------------------------------------------------
# Pi5: scan form of Q_alpha^{-1}, independent of any time DFT
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("Nt,alpha", [(8, 1e-2), (16, 1e-3), (32, 1e-4)])
def test_precond_apply_equals_scan_form(Nt, alpha):
    st = O.Setup(2, 8, Nt, 1.0 / Nt, alpha, a=0.05)
    rng = np.random.default_rng(9)
    R = rng.standard_normal((Nt, 8, 8))
    Rh = np.fft.fftn(R, axes=(1, 2))
    z = np.zeros_like(Rh)
    acc = np.zeros_like(Rh[0])
    for m in range(Nt):
        acc = Rh[m] + st.E * acc
        z[m] = acc
    ET = st.E ** Nt
    Sh = np.array([z[m] + alpha * st.E ** (m + 1) * z[-1] / (1 - alpha * ET)
                   for m in range(Nt)])
    S_scan = np.fft.ifftn(Sh, axes=(1, 2)).real
    S = O.precond_apply(st, R)
    # roundoff of the diagonalisation grows like eps/alpha
    assert np.max(np.abs(S - S_scan)) < 50 * 2.2e-16 / alpha * np.max(
        np.abs(S_scan))


# ---------------------------------------------------------------------------
# Pi6: GMRES -- finite termination (thm_gmres1), Elman-type bound
# (gmres3_thm), and agreement with scipy
# ---------------------------------------------------------------------------
def test_gmres_finite_termination():
    n, Nt = 6, 5
    st = O.Setup(1, n, Nt, 0.1, 0.3, a=0.5, c=0.1)
    u0 = _field(np.random.default_rng(8), 1, n)
    U, it, hist = O.gmres_solve(st, u0, restart=50, tol=1e-13, max_iter=50)
    assert it <= n + 1
    assert O.rel_err(U, O.dense_solve(st, u0)) < 1e-11


@pytest.mark.parametrize("alpha", [0.02, 0.1])
def test_gmres_residual_bound(alpha):
    Nt = 8
    assert alpha < 2 / (3 + math.sqrt(Nt))
    st = O.Setup(1, 16, Nt, 0.1, alpha, a=0.3, c=0.0)
    u0 = _field(np.random.default_rng(12), 1, 16)
    _, it, hist = O.gmres_solve(st, u0, restart=100, tol=1e-14, max_iter=30)
    rate = math.sqrt(4 * alpha * (1 - alpha))
    for k, r in enumerate(hist):
        assert r <= rate ** k * hist[0] * (1 + 1e-8) + 1e-15


def test_gmres_matches_scipy():
    st = O.Setup(1, 12, 6, 0.1, 0.05, a=0.5)
    u0 = _field(np.random.default_rng(13), 1, 12)
    D = O.dense_operators(st)
    M = np.linalg.solve(D["Qa"], D["Q"])
    f = np.zeros(72)
    f[:12] = D["A"] @ u0
    b = np.linalg.solve(D["Qa"], f)
    xs, info = scipy.sparse.linalg.gmres(M, b, rtol=1e-13, restart=20,
                                         maxiter=100)
    U, it, _ = O.gmres_solve(st, u0, restart=20, tol=1e-13)
    assert info == 0
    assert np.max(np.abs(U.ravel() - xs)) < 1e-11


# ---------------------------------------------------------------------------
# Pi7: nonlinear schemes -- closed form for N(u) = beta u, convergence order,
# fixed point and Newton-GMRES reach the unique all-at-once solution
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", [1, 2])
def test_linear_reaction_closed_form(scheme):
    beta = 0.7
    n, Nt, dt = 16, 10, 0.05
    st = O.Setup(1, n, Nt, dt, 1e-2, a=0.2, n1=beta, scheme=scheme)
    u0 = _field(np.random.default_rng(6), 1, n)
    U = O.sequential(st, u0)
    k = np.fft.fftfreq(n, 1.0 / n)
    mu = -0.2 * k * k
    z = dt * mu
    # independent phi evaluations (mpmath)
    p1 = np.array([float(_mp_phi1(v)) for v in z])
    p2 = np.array([float(_mp_phi2(v)) for v in z])
    E = np.exp(z)
    u0h = np.fft.fft(u0)
    if scheme == 1:
        g = E + dt * p1 * beta
        pred = [g ** (m + 1) * u0h for m in range(Nt)]
    else:
        # u_n = (E + dt(p1+p2)beta) u_{n-1} - dt p2 beta u_{n-2}, u_{-1}=u_0
        c1 = E + dt * (p1 + p2) * beta
        c2 = -dt * p2 * beta
        prev2, prev, pred = u0h, u0h, []
        for m in range(Nt):
            nxt = c1 * prev + c2 * prev2
            pred.append(nxt)
            prev2, prev = prev, nxt
    got = np.fft.fft(U, axis=1)
    assert np.max(np.abs(got - np.array(pred))) < 1e-13


@pytest.mark.parametrize("scheme,order", [(1, 1.0), (2, 2.0)])
def test_convergence_order(scheme, order):
    """Observed order against the exact solution of u_t = a u_xx + beta u
    (beta linear so the exact flow is known): ETD1 first, ETD2 second."""
    n, T, beta, a = 16, 1.0, 1.5, 0.1
    x = 2 * np.pi * np.arange(n) / n
    u0 = np.sin(x) + 0.5 * np.cos(2 * x)
    exact = np.exp((-a + beta) * T) * np.sin(x) \
        + 0.5 * np.exp((-4 * a + beta) * T) * np.cos(2 * x)
    errs = []
    for Nt in (16, 32, 64, 128):
        st = O.Setup(1, n, Nt, T / Nt, 1e-2, a=a, n1=beta, scheme=scheme)
        errs.append(np.max(np.abs(O.sequential(st, u0)[-1] - exact)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert abs(rates[-1] - order) < 0.1, rates


@pytest.mark.parametrize("scheme", [1, 2])
def test_nonlinear_fixed_point_reaches_sequential(scheme):
    inst = W.scaled(W.allen_cahn2d(scheme=scheme), n=16, Nt=16)
    st = O.Setup.from_instance(inst)
    ref = O.sequential(st, inst.u0)
    U, it, _ = O.fixed_point(st, inst.u0, tol=1e-13, max_iter=200)
    assert O.rel_err(U, ref) < 1e-12


@pytest.mark.parametrize("scheme", [1, 2])
def test_newton_gmres_reaches_sequential(scheme):
    inst = W.scaled(W.rd2d(), n=16, Nt=16)
    inst.scheme = scheme
    st = O.Setup.from_instance(inst)
    ref = O.sequential(st, inst.u0)
    U, steps, inner, hist = O.newton_gmres(st, inst.u0, tol=1e-12)
    assert O.rel_err(U, ref) < 1e-10
    assert steps <= 10


# ---------------------------------------------------------------------------
# G'(U): the derivative of the lagged nonlinear term (Newton's Jacobian of
# Sec. 5, eq. newton_2, for the ETD schemes), against differences of G
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme,dim,n,Nt", [(1, 1, 16, 6), (2, 1, 16, 6),
                                             (1, 2, 8, 5), (2, 2, 8, 5),
                                             (2, 3, 4, 4)])
def test_gprime_equals_richardson_difference(scheme, dim, n, Nt):
    """N(u) = n1 u + n2 u^2 + n3 u^3 is a cubic polynomial, so the lagged
    term G(U) (plus the constant u_0 part of f) is cubic in U.  For a cubic
    the central difference D(h) = [G(U + hV) - G(U - hV)] / (2h) equals
    G'(U)V + h^2/6 G'''(U)[V,V,V] exactly, so the Richardson combination
    (4 D(h) - D(2h)) / 3 is G'(U)V with no truncation error at all: the
    only difference left is rounding (about eps |G| / h)."""
    st = O.Setup(dim, n, Nt, 0.05, 1e-2, a=0.1, n1=1.0, n2=0.3, n3=-1.0,
                 scheme=scheme)
    rng = np.random.default_rng([dim, n, Nt, scheme])
    u0 = _field(rng, dim, n)
    U = rng.uniform(-0.9, 0.9, size=(Nt,) + (n,) * dim)
    V = rng.uniform(-1.0, 1.0, size=U.shape)
    h = 1e-2

    def D(s):
        return (O.nonlinear_term(st, u0, U + s * V)
                - O.nonlinear_term(st, u0, U - s * V)) / (2.0 * s)
    fd = (4.0 * D(h) - D(2.0 * h)) / 3.0
    got = O.gprime_apply(st, u0, U, V)
    assert np.max(np.abs(got - fd)) <= 1e-11 * np.max(np.abs(fd))
    # the first slice depends on u_0 only: its row of G' is zero
    assert np.max(np.abs(got[0])) == 0.0


def test_gprime_linear_reaction_is_scaled_shift():
    """N(u) = beta u: G(U) is linear, G'(U)V = G(V) - G(0) for any U, and
    per Fourier mode slice n of G'V is dt phi1 beta v_{n-1} (ETD1) or
    dt[(phi1 + phi2) beta v_{n-1} - phi2 beta v_{n-2}] (ETD2), v_0 = v_{-1}
    = 0, with phi from mpmath (independent of the oracle's phi)."""
    beta, n, Nt, dt = 0.7, 16, 6, 0.05
    rng = np.random.default_rng(11)
    k = np.fft.fftfreq(n, 1.0 / n)
    z = dt * (-0.2 * k * k)
    p1 = np.array([float(_mp_phi1(v)) for v in z])
    p2 = np.array([float(_mp_phi2(v)) for v in z])
    for scheme in (1, 2):
        st = O.Setup(1, n, Nt, dt, 1e-2, a=0.2, n1=beta, scheme=scheme)
        U = rng.uniform(-0.9, 0.9, size=(Nt, n))
        V = rng.uniform(-1.0, 1.0, size=(Nt, n))
        got = np.fft.fft(O.gprime_apply(st, U[0], U, V), axis=1)
        Vh = np.fft.fft(V, axis=1)
        pred = np.zeros_like(Vh)
        for m in range(1, Nt):
            if scheme == 1:
                pred[m] = dt * p1 * beta * Vh[m - 1]
            else:
                prev2 = Vh[m - 2] if m >= 2 else 0.0
                pred[m] = dt * ((p1 + p2) * beta * Vh[m - 1]
                                - p2 * beta * prev2)
        assert np.max(np.abs(got - pred)) < 1e-13


# ---------------------------------------------------------------------------
# the error metric of Sec. 6: L_inf(0,T; L2), normalised
# ---------------------------------------------------------------------------
def test_rel_err_hand_computed():
    """Two slices of two points.  U - V has slice norms 5 (3, 4) and 1
    (1, 0); V has slice norms 10 (0, 10) and 1 (0, 1): the L_inf(0,T;L2)
    ratio is 5/10 = 0.5.  A Frobenius ratio would give sqrt(26/101) = 0.507,
    an entrywise max ratio 4/10, a mean over slices 3/5.5, normalising by U
    instead of V 5/sqrt(9 + 196)."""
    V = np.array([[0.0, 10.0], [0.0, 1.0]])
    U = V + np.array([[3.0, 4.0], [1.0, 0.0]])
    assert O.rel_err(U, V) == pytest.approx(0.5, rel=1e-15)
    # complex entries: |3i| and |4| form the same slice norm
    Vc = V.astype(complex)
    Uc = Vc + np.array([[3j, 4.0], [-1j, 0.0]])
    assert O.rel_err(Uc, Vc) == pytest.approx(0.5, rel=1e-15)
    # 2D slices: the slice norm runs over every spatial point
    V2 = np.zeros((3, 2, 2))
    V2[1, 0, 1] = 2.0
    U2 = V2.copy()
    U2[2] = [[1.0, 1.0], [1.0, 1.0]]    # slice norm 2
    U2[0, 1, 1] = 1.0                   # slice norm 1
    assert O.rel_err(U2, V2) == pytest.approx(1.0, rel=1e-15)
