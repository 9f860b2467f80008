"""Pins of the oracle with complex symbols: periodic advection-diffusion
L = a Lap - b.grad - c (the remark after Theorem thm_gmres22), whose symbol
mu_k = -a|k|^2 - c - i b.k' makes E_k = e^{dt mu_k} complex while the state
stays real.

The second half covers complex states: the Schroedinger equation of Sec. 6
(a = i, c = 2i), whose symbol is purely imaginary.

Independent references: the exact solution of the PDE for trigonometric
data (advected, damped or rotating modes), norm conservation, the per-mode
closed form of every iterate
with a complex e^{mu T} (derived from the iteration matrix of eq.
pcond_system, as for real symbols), dense LU and dense eigenvalues on the
assembled matrices, and GMRES's finite termination.
"""
import math

import numpy as np
import pytest

import oracle as O


def _field(rng, dim, n):
    return rng.uniform(-0.9, 0.9, size=(n,) * dim)


def test_advection_diffusion_exact_solution_1d():
    """u_t = a u_xx - b u_x from trigonometric data: each mode moves with
    speed b and decays by e^{-a k^2 t}; ETD1 is exact in time here."""
    n, Nt, T, a, b = 32, 16, 1.0, 0.1, 2.0
    st = O.Setup(1, n, Nt, T / Nt, 1e-2, a=a, b=(b, 0.0, 0.0))
    x = 2 * np.pi * np.arange(n) / n
    u0 = np.sin(x) + 0.3 * np.cos(3 * x) - 0.2 * np.sin(7 * x)
    U = O.sequential(st, u0)
    for m in range(Nt):
        t = (m + 1) * T / Nt
        ex = (np.exp(-a * t) * np.sin(x - b * t)
              + 0.3 * np.exp(-9 * a * t) * np.cos(3 * (x - b * t))
              - 0.2 * np.exp(-49 * a * t) * np.sin(7 * (x - b * t)))
        assert np.max(np.abs(U[m] - ex)) < 1e-14
    Uf, _, _ = O.fixed_point(st, u0, tol=1e-15, max_iter=40)
    assert O.rel_err(Uf, U) < 1e-14


def test_advection_2d_exact_solution():
    n, Nt, T, a, b = 16, 8, 0.5, 0.05, (1.5, -0.7)
    st = O.Setup(2, n, Nt, T / Nt, 1e-3, a=a, c=0.2, b=b + (0.0,))
    x = 2 * np.pi * np.arange(n) / n
    X, Y = np.meshgrid(x, x, indexing="ij")
    u0 = np.cos(2 * X + Y)
    U = O.sequential(st, u0)
    for m in range(Nt):
        t = (m + 1) * T / Nt
        ex = np.exp(-(5 * a + 0.2) * t) * np.cos(
            2 * (X - b[0] * t) + (Y - b[1] * t))
        assert np.max(np.abs(U[m] - ex)) < 1e-14


def test_complex_symbol_is_hermitian():
    """E_{-k} = conj(E_k), Nyquist included: A maps real fields to real
    fields, so no imaginary part is discarded."""
    st = O.Setup(2, 8, 4, 0.1, 1e-2, a=0.3, b=(1.0, -2.0, 0.0))
    E = st.E
    flip = E[np.ix_(-np.arange(8) % 8, -np.arange(8) % 8)]
    assert np.max(np.abs(flip - np.conj(E))) < 1e-15
    rng = np.random.default_rng(3)
    v = rng.standard_normal((8, 8))
    Av = st.spectral_apply(v, E)
    assert np.max(np.abs(Av.imag)) < 1e-15


@pytest.mark.parametrize("dim,n,Nt,alpha,a,b", [
    (1, 16, 8, 1e-2, 0.1, (2.0, 0, 0)),
    (2, 8, 8, 0.2, 0.05, (1.0, 0.5, 0)),
    (1, 32, 16, 1e-3, 1e-5, (2.0, 0, 0)),   # advection dominated
])
def test_complex_symbol_iterates_closed_form(dim, n, Nt, alpha, a, b):
    """Every linear iterate from U^0 = 0: u^_{n,k}^k = (1 - psi_k^k) E_k^n
    u^_{0,k}, psi_k = -alpha e^{mu_k T}/(1 - alpha e^{mu_k T}), now with a
    complex e^{mu_k T}."""
    st = O.Setup(dim, n, Nt, 1.0 / Nt, alpha, a=a, b=b)
    u0 = _field(np.random.default_rng(7), dim, n)
    _, _, (_, its) = O.fixed_point(st, u0, max_iter=4, tol=0.0, record=True)
    axes = tuple(range(dim))
    u0h = np.fft.fftn(u0, axes=axes)
    ET = st.E ** Nt
    psi = -alpha * ET / (1.0 - alpha * ET)
    for k, Uk in enumerate(its, start=1):
        for m in range(Nt):
            pred = (1.0 - psi ** k) * st.E ** (m + 1) * u0h
            got = np.fft.fftn(Uk[m], axes=axes)
            assert np.max(np.abs(got - pred)) <= 1e-13 * np.max(np.abs(u0h))


@pytest.mark.parametrize("a", [0.1, 1e-5])
def test_complex_symbol_preconditioned_spectrum(a):
    """eig(Q_alpha^{-1} Q) = {1} u {1/(1 - alpha e^{mu_k T})}: complex now,
    still within alpha/(1 - alpha) of 1 (the remark after thm_gmres22)."""
    st = O.Setup(1, 8, 5, 0.1, 0.05, a=a, b=(2.0, 0.0, 0.0))
    D = O.dense_operators(st)
    ev = np.linalg.eigvals(np.linalg.solve(D["Qa"], D["Q"]))
    ET = st.E ** st.Nt
    pred = np.concatenate([np.ones(8 * 4), 1.0 / (1.0 - st.alpha * ET)])
    assert np.allclose(np.sort_complex(ev), np.sort_complex(pred + 0j),
                       atol=1e-10)
    assert np.max(np.abs(ev - 1)) <= st.alpha / (1 - st.alpha) + 1e-12
    assert np.max(np.abs(np.imag(1.0 / (1.0 - st.alpha * ET)))) > 1e-4


@pytest.mark.parametrize("dim,n,Nt,alpha", [(1, 12, 8, 1e-2), (2, 4, 4, 0.3)])
def test_complex_symbol_precond_equals_dense_inverse(dim, n, Nt, alpha):
    st = O.Setup(dim, n, Nt, 0.1, alpha, a=0.4, b=(1.3, -0.6, 0.0))
    D = O.dense_operators(st)
    assert np.max(np.abs(D["A"] - D["A"].real)) == 0.0
    R = np.random.default_rng(5).standard_normal((Nt,) + (n,) * dim)
    S = O.precond_apply(st, R)
    Sd = np.linalg.solve(D["Qa"], R.ravel()).reshape(R.shape)
    assert np.max(np.abs(S - Sd)) < 1e-12 * np.max(np.abs(Sd))
    u0 = _field(np.random.default_rng(6), dim, n)
    assert O.rel_err(O.sequential(st, u0), O.dense_solve(st, u0, D)) < 1e-14


def test_complex_symbol_gmres_finite_termination():
    n, Nt = 6, 5
    st = O.Setup(1, n, Nt, 0.1, 0.3, a=0.5, c=0.1, b=(2.0, 0.0, 0.0))
    u0 = _field(np.random.default_rng(8), 1, n)
    U, it, _ = O.gmres_solve(st, u0, restart=50, tol=1e-13, max_iter=50)
    assert it <= n + 1
    assert O.rel_err(U, O.sequential(st, u0)) < 1e-11


@pytest.mark.parametrize("scheme", [1, 2])
def test_complex_symbol_nonlinear_dense_newton(scheme):
    """Allen-Cahn with advection: sequential ETD1/ETD2 stepping with complex
    phi weights equals the dense Newton solution of the all-at-once system."""
    st = O.Setup(1, 8, 6, 0.05, 1e-2, a=0.3, n1=1.0, n3=-1.0, scheme=scheme,
                 b=(1.5, 0.0, 0.0))
    u0 = _field(np.random.default_rng(4), 1, 8)
    assert O.rel_err(O.sequential(st, u0), O.dense_newton(st, u0)) < 1e-13
    U, _, _ = O.fixed_point(st, u0, tol=1e-15, max_iter=80)
    assert O.rel_err(U, O.sequential(st, u0)) < 1e-13


def test_complex_phi_against_series():
    """phi1, phi2 for complex z against their power series summed in
    extended precision (Python complex with many terms, small |z|) and the
    closed forms at larger |z|."""
    zs = np.array([1e-9j, 0.3 + 0.4j, -2.0 + 5.0j, -30.0 - 2.0j, 0.5j])
    p1 = O.phi1(zs)
    p2 = O.phi2(zs)
    for z, a1, a2 in zip(zs, p1, p2):
        z = complex(z)
        if abs(z) < 1:
            s1 = sum(z ** j / math.factorial(j + 1) for j in range(40))
            s2 = sum(z ** j / math.factorial(j + 2) for j in range(40))
        else:
            import cmath
            s1 = (cmath.exp(z) - 1) / z
            s2 = (cmath.exp(z) - 1 - z) / (z * z)
        assert abs(a1 - s1) <= 1e-15 * abs(s1)
        assert abs(a2 - s2) <= 1e-15 * abs(s2)


# ---------------------------------------------------------------------------
# complex state: the Schroedinger equation of Sec. 6 (a = i, c = i c_im)
# ---------------------------------------------------------------------------
def _schroedinger(dim, n, Nt, T, alpha, c_im=2.0, scheme=1):
    return O.Setup(dim, n, Nt, T / Nt, alpha, a=0.0, a_im=1.0, c_im=c_im,
                   scheme=scheme)


def _packet(dim, n, k0=5.0, w=0.4):
    x = 2 * np.pi * np.arange(n) / n
    g = np.meshgrid(*([x] * dim), indexing="ij")
    r2 = sum((gi - np.pi) ** 2 for gi in g)
    return np.exp(-r2 / (2 * w * w)) * np.exp(-1j * k0 * (g[0] - np.pi))


@pytest.mark.parametrize("scheme", [1, O.EBDF2])
def test_schroedinger_plane_waves_exact(scheme):
    """u_t = i u_xx - 2i u from e^{i3x} + 0.5 e^{-2ix}: each plane wave
    rotates by e^{-i(k^2 + 2)t}; ETD1 and EBDF2 (from u_1 = A u_0) are exact."""
    n, Nt, T = 32, 16, 1.0
    st = _schroedinger(1, n, Nt, T, 1e-2, scheme=scheme)
    x = 2 * np.pi * np.arange(n) / n
    u0 = np.exp(3j * x) + 0.5 * np.exp(-2j * x)
    t = (np.arange(Nt) + 1) * T / Nt
    ex = np.array([np.exp(-11j * tt) * np.exp(3j * x)
                   + 0.5 * np.exp(-6j * tt) * np.exp(-2j * x) for tt in t])
    assert np.max(np.abs(O.sequential(st, u0) - ex)) < 1e-14
    U, _, _ = O.fixed_point(st, u0, tol=1e-15, max_iter=40)
    assert np.max(np.abs(U - ex)) < 1e-13


def test_schroedinger_conserves_norm():
    """i Lap - 2i has a purely imaginary spectrum: A is unitary, so every
    slice keeps the l2 norm of u_0."""
    st = _schroedinger(2, 16, 8, 0.5, 1e-3)
    u0 = _packet(2, 16)
    U = O.sequential(st, u0)
    n0 = np.linalg.norm(u0)
    for m in range(st.Nt):
        assert abs(np.linalg.norm(U[m]) - n0) < 1e-13 * n0


def test_schroedinger_iterates_closed_form():
    """Every iterate: (1 - psi_k^k) E_k^n u^_{0,k} with |e^{mu_k T}| = 1, so
    |psi_k| = alpha/|1 - alpha e^{mu_k T}| for every mode."""
    st = _schroedinger(1, 16, 8, 1.0, 0.05)
    u0 = _packet(1, 16, k0=3.0, w=0.6)
    _, _, (_, its) = O.fixed_point(st, u0, max_iter=4, tol=0.0, record=True)
    u0h = np.fft.fft(u0)
    ET = st.E ** st.Nt
    assert np.allclose(np.abs(ET), 1.0, atol=1e-14)
    psi = -st.alpha * ET / (1.0 - st.alpha * ET)
    for k, Uk in enumerate(its, start=1):
        for m in range(st.Nt):
            pred = (1.0 - psi ** k) * st.E ** (m + 1) * u0h
            assert np.max(np.abs(np.fft.fft(Uk[m]) - pred)) <= \
                1e-13 * np.max(np.abs(u0h))


def test_schroedinger_precond_and_solve_dense():
    st = _schroedinger(1, 8, 5, 0.5, 0.1)
    D = O.dense_operators(st)
    rng = np.random.default_rng(12)
    R = rng.standard_normal((5, 8)) + 1j * rng.standard_normal((5, 8))
    S = O.precond_apply(st, R)
    Sd = np.linalg.solve(D["Qa"], R.ravel()).reshape(R.shape)
    assert np.max(np.abs(S - Sd)) < 1e-12 * np.max(np.abs(Sd))
    u0 = _packet(1, 8, w=0.8)
    assert O.rel_err(O.sequential(st, u0), O.dense_solve(st, u0, D)) < 1e-14
    ev = np.linalg.eigvals(np.linalg.solve(D["Qa"], D["Q"]))
    assert np.max(np.abs(ev - 1)) <= st.alpha / (1 - st.alpha) + 1e-12


def test_schroedinger_gmres_finite_termination():
    """Real GMRES on the real and imaginary parts: the preconditioned
    operator is the identity plus a real rank of 2 per excited mode."""
    n, Nt = 6, 5
    st = _schroedinger(1, n, Nt, 0.5, 0.3)
    u0 = _packet(1, n, w=0.9)
    U, it, _ = O.gmres_solve(st, u0, restart=50, tol=1e-13, max_iter=50)
    assert it <= 2 * n + 1
    assert O.rel_err(U, O.sequential(st, u0)) < 1e-11
    x = 2 * np.pi * np.arange(16) / 16
    st1 = _schroedinger(1, 16, 8, 1.0, 0.1)
    U1, it1, _ = O.gmres_solve(st1, np.exp(3j * x), restart=20, tol=1e-12)
    assert it1 <= 3
