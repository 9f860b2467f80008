"""Pins of the oracle's EBDF2 path (second-order exponential BDF, Sec. 4).

Each check compares the oracle with something independent of it: the closed
form A^n u_0 that the recurrence reaches from u_1 = A u_0, dense LU on the
all-at-once matrices assembled entry by entry, the diagonalisation of the
alpha-circulants C_0^alpha and C_1^alpha, the exact spectrum of the
iteration matrix (Theorem thm_bdf2), the clustering radius of the
preconditioned spectrum (Lemma gmres_centered_at1_2nd_order) and GMRES's
finite termination (Theorem thm_gmres1_2ndorder).
"""
import math

import numpy as np
import pytest

import oracle as O


def _field(rng, dim, n):
    return rng.uniform(-0.9, 0.9, size=(n,) * dim)


def _setup(dim, n, Nt, alpha, a=0.4, c=0.0, dt=0.1):
    return O.Setup(dim, n, Nt, dt, alpha, a=a, c=c, scheme=O.EBDF2)


# ---------------------------------------------------------------------------
# the recurrence from u_1 = A u_0 reproduces A^n u_0 (4/3 - 1/3 = 1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n,Nt", [(1, 16, 8), (2, 8, 16), (3, 4, 5)])
def test_ebdf2_sequential_closed_form(dim, n, Nt):
    st = _setup(dim, n, Nt, 1e-2, a=0.3, c=0.1)
    u0 = _field(np.random.default_rng(21), dim, n)
    U = O.sequential_ebdf2(st, u0)
    axes = tuple(range(dim))
    u0h = np.fft.fftn(u0, axes=axes)
    for m in range(Nt):
        got = np.fft.fftn(U[m], axes=axes)
        assert np.max(np.abs(got - st.E ** (m + 1) * u0h)) <= \
            1e-14 * np.max(np.abs(u0h))


def test_ebdf2_single_mode_heat_exact():
    n, Nt, T = 16, 8, 1.0
    st = O.Setup(1, n, Nt, T / Nt, 1e-2, a=1.0, scheme=O.EBDF2)
    x = 2 * np.pi * np.arange(n) / n
    u0 = np.sin(x)
    exact = np.array([np.exp(-(k + 1) * T / Nt) * np.sin(x)
                      for k in range(Nt)])
    assert np.max(np.abs(O.sequential_ebdf2(st, u0) - exact)) < 1e-15
    U, it, _ = O.fixed_point(st, u0, tol=1e-15, max_iter=30)
    assert np.max(np.abs(U - exact)) < 1e-15


# ---------------------------------------------------------------------------
# dense assembled R, R_alpha (eqs. all_at_once_2ndorder, pcond-2nd-order)
# ---------------------------------------------------------------------------
def _dense_f2(D, u0, Nt):
    A, B = D["A"], D["B"]
    Ns = A.shape[0]
    u1 = A @ u0.ravel()
    f2 = np.zeros((Nt - 1) * Ns)
    f2[:Ns] = 4.0 / 3.0 * A @ u1 - 1.0 / 3.0 * B @ u0.ravel()
    f2[Ns:2 * Ns] = -1.0 / 3.0 * B @ u1
    return f2


@pytest.mark.parametrize("dim,n,Nt", [(1, 8, 6), (1, 12, 9), (2, 4, 5)])
def test_ebdf2_dense_lu_equals_sequential(dim, n, Nt):
    st = _setup(dim, n, Nt, 1e-2, a=0.7, c=0.05)
    u0 = _field(np.random.default_rng(22), dim, n)
    D = O.dense_operators_ebdf2(st)
    v = np.linalg.solve(D["R"], _dense_f2(D, u0, Nt))
    U = O.sequential_ebdf2(st, u0)
    assert np.max(np.abs(v - U[1:].ravel())) < 1e-14 * np.max(np.abs(U))


def test_ebdf2_residual_and_operators_equal_dense():
    Nt, n = 7, 8
    st = _setup(1, n, Nt, 0.05, a=0.9)
    D = O.dense_operators_ebdf2(st)
    rng = np.random.default_rng(23)
    u0 = _field(rng, 1, n)
    U = rng.standard_normal((Nt, n))
    R = O.residual_ebdf2(st, u0, U)
    assert np.allclose(R[0], D["A"] @ u0 - U[0], atol=1e-14)
    want = _dense_f2(D, u0, Nt) - D["R"] @ U[1:].ravel()
    assert np.allclose(R[1:].ravel(), want, atol=1e-13)
    V = U[1:]
    assert np.allclose(O.r_apply_ebdf2(st, V).ravel(), D["R"] @ V.ravel(),
                       atol=1e-13)
    assert np.allclose(O.ralpha_apply_ebdf2(st, V).ravel(),
                       D["Ra"] @ V.ravel(), atol=1e-13)


@pytest.mark.parametrize("dim,n,Nt,alpha", [(1, 12, 8, 1e-2), (2, 4, 5, 0.3),
                                            (1, 8, 9, 1e-3)])
def test_ebdf2_precond_equals_dense_inverse(dim, n, Nt, alpha):
    st = _setup(dim, n, Nt, alpha, a=0.4)
    D = O.dense_operators_ebdf2(st)
    rng = np.random.default_rng(24)
    R = rng.standard_normal((Nt,) + (n,) * dim)
    S = O.precond_apply_ebdf2(st, R)
    assert np.array_equal(S[0], R[0])
    Sd = np.linalg.solve(D["Ra"], R[1:].ravel())
    assert np.max(np.abs(S[1:].ravel() - Sd)) < 1e-12 * np.max(np.abs(Sd))


@pytest.mark.parametrize("Nt,alpha", [(5, 0.3), (8, 1e-2), (17, 1e-3)])
def test_ebdf2_alpha_circulants_share_eigenvectors(Nt, alpha):
    """C_0^alpha = P D_0 P^{-1} and C_1^alpha = P D_1 P^{-1} with
    P = Gamma_alpha^{-1} F^* on Nt-1 points (Sec. 4)."""
    st = _setup(1, 4, Nt, alpha)
    gamma, lam0, lam1 = O.ebdf2_tables(st)
    N = Nt - 1
    omega = np.exp(2j * np.pi / N)
    l = np.arange(N)
    F = omega ** np.outer(l, l) / np.sqrt(N)
    P = np.diag(1.0 / gamma) @ F.conj().T
    Pi = np.linalg.inv(P)
    D = O.dense_operators_ebdf2(st)
    assert np.max(np.abs(P @ np.diag(lam0) @ Pi - D["C0a"])) < 1e-12
    assert np.max(np.abs(P @ np.diag(lam1) @ Pi - D["C1a"])) < 1e-12
    # C_1 is the second sub-diagonal, and C_1^alpha the square of C_0^alpha
    assert np.array_equal(D["C1"], np.diag(np.ones(N - 2), -2))
    assert np.allclose(D["C1a"], D["C0a"] @ D["C0a"], atol=1e-15)


# ---------------------------------------------------------------------------
# Theorem thm_bdf2: exact spectrum of I - R_alpha^{-1} R
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("Nt,alpha,c", [(6, 0.05, 0.0), (8, 0.2, 0.3),
                                        (5, 1e-2, 0.1)])
def test_ebdf2_iteration_matrix_spectrum(Nt, alpha, c):
    n = 6
    st = _setup(1, n, Nt, alpha, a=0.5, c=c)
    D = O.dense_operators_ebdf2(st)
    M = np.eye(D["R"].shape[0]) - np.linalg.solve(D["Ra"], D["R"])
    ev = np.linalg.eigvals(M)
    N = Nt - 1
    pred = []
    for E in st.E:                       # one spatial mode each
        y1 = alpha * E ** N
        y2 = alpha * (E / 3.0) ** N
        pred += [-y1 / (1 - y1), -y2 / (1 - y2)] + [0.0] * (N - 2)
    pred = np.sort_complex(np.array(pred) + 0j)
    got = np.sort_complex(ev)
    # the zero eigenvalue is defective, so its computed copies scatter
    big = np.abs(pred) > 1e-3 * alpha ** N
    assert np.allclose(np.sort(np.abs(got))[::-1][:big.sum()],
                       np.sort(np.abs(pred[big]))[::-1], rtol=1e-6)
    assert np.max(np.abs(ev)) <= alpha / (1 - alpha) * (1 + 1e-9)


@pytest.mark.parametrize("alpha", [0.05, 0.2])
def test_ebdf2_preconditioned_spectrum_cluster(alpha):
    """Lemma gmres_centered_at1_2nd_order: eigenvalues of R_alpha^{-1} R lie
    within (alpha + alpha^2)/(1 - alpha - alpha^2) of 1."""
    st = _setup(1, 8, 7, alpha, a=0.3)
    D = O.dense_operators_ebdf2(st)
    ev = np.linalg.eigvals(np.linalg.solve(D["Ra"], D["R"]))
    eps0 = (alpha + alpha ** 2) / (1 - alpha - alpha ** 2)
    assert np.max(np.abs(ev - 1)) <= eps0


# ---------------------------------------------------------------------------
# fixed point and GMRES
# ---------------------------------------------------------------------------
def test_ebdf2_fixed_point_rate_is_theorem_radius():
    """With the mean mode present and c = 0 the dominant eigenvalue of the
    iteration matrix is -alpha/(1 - alpha) (E = 1 at k = 0), so successive
    errors shrink by that factor."""
    alpha = 0.05
    # every other mode contracts by at most alpha e^{-2}/(1 - alpha e^{-2})
    # (a dt N = 2), and with N = 4 the nilpotent part of the iteration
    # matrix is gone after two iterations
    st = _setup(1, 16, 5, alpha, a=0.5, dt=1.0)
    u0 = 0.4 + _field(np.random.default_rng(25), 1, 16)
    ref = O.sequential_ebdf2(st, u0)
    _, _, (hist, its) = O.fixed_point(st, u0, max_iter=6, tol=0.0,
                                      record=True)
    errs = [np.linalg.norm(U - ref) for U in its]
    rho = alpha / (1 - alpha)
    for k in (3, 4, 5):
        assert abs(errs[k] / errs[k - 1] - rho) < 1e-3 * rho


@pytest.mark.parametrize("dim,n,Nt,alpha", [(1, 16, 8, 1e-2),
                                            (2, 8, 16, 1e-3)])
def test_ebdf2_fixed_point_reaches_closed_form(dim, n, Nt, alpha):
    st = _setup(dim, n, Nt, alpha, a=0.2, dt=1.0 / Nt)
    u0 = _field(np.random.default_rng(26), dim, n)
    ref = O.sequential_ebdf2(st, u0)
    U, it, _ = O.fixed_point(st, u0, ref=ref, ref_tol=1e-13, max_iter=40)
    assert O.rel_err(U, ref) <= 1e-13
    # contraction alpha/(1-alpha) per iteration bounds the count
    assert it <= math.ceil(math.log(1e-13) / math.log(alpha / (1 - alpha))) + 2


def test_ebdf2_gmres_finite_termination():
    """Theorem thm_gmres1_2ndorder: at most 2 Nx + 1 iterations."""
    n, Nt = 6, 7
    st = _setup(1, n, Nt, 0.3, a=0.5, c=0.1)
    u0 = _field(np.random.default_rng(27), 1, n)
    U, it, _ = O.gmres_solve_ebdf2(st, u0, restart=60, tol=1e-13,
                                   max_iter=60)
    assert it <= 2 * n + 1
    assert O.rel_err(U, O.sequential_ebdf2(st, u0)) < 1e-11


def test_ebdf2_gmres_single_mode_three_steps():
    """u_0 = sin x excites one |k|: R_alpha^{-1} R restricted to it is
    identity plus rank two, so GMRES stops within three iterations."""
    n, Nt = 16, 8
    st = _setup(1, n, Nt, 0.1, a=1.0)
    x = 2 * np.pi * np.arange(n) / n
    U, it, _ = O.gmres_solve_ebdf2(st, np.sin(x), restart=20, tol=1e-12,
                                   max_iter=20)
    assert it <= 3
    assert O.rel_err(U, O.sequential_ebdf2(st, np.sin(x))) < 1e-12
