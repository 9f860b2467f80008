"""Pins of the oracle's IF1 path (the implicit integrating-factor scheme of
Sec. 5, u_n = A u_{n-1} + dt N(u_n)).

Independent references: dense Newton on the assembled all-at-once system,
the closed form of the scheme for a linear reaction N(u) = beta u, the
closed form of every preconditioned iterate in that case (the iteration is
then the linear one with E/(1 - dt beta)), and the contraction of Theorem
thm_nonlin for the paper's outer iteration with exact inner solves, with the
factor e^{-TM/(1 + 2 dt M)} that its proof gives for the norm.
"""
import math

import numpy as np
import pytest

import oracle as O


def _setup(dim, n, Nt, dt, alpha, jac=1, a=0.3, c=0.0, n1=1.0, n2=0.0,
           n3=-1.0):
    return O.Setup(dim, n, Nt, dt, alpha, a=a, c=c, n1=n1, n2=n2, n3=n3,
                   scheme=O.IF1, jac=jac)


def _field(rng, dim, n, amp=0.9):
    return rng.uniform(-amp, amp, size=(n,) * dim)


@pytest.mark.parametrize("dim,n,Nt", [(1, 8, 6), (2, 4, 4)])
@pytest.mark.parametrize("n2", [0.0, -0.4])
def test_if1_sequential_equals_dense_newton(dim, n, Nt, n2):
    st = _setup(dim, n, Nt, 0.05, 1e-2, n2=n2)
    u0 = _field(np.random.default_rng(31), dim, n)
    Ud = O.dense_newton_if1(st, u0, tol=1e-15)
    assert O.rel_err(O.sequential_if1(st, u0), Ud) < 1e-14


@pytest.mark.parametrize("beta", [-2.0, 0.7])
def test_if1_linear_reaction_closed_form(beta):
    """N(u) = beta u: (1 - dt beta) u_n = A u_{n-1}, so
    u^_{n,k} = (E_k / (1 - dt beta))^n u^_{0,k}."""
    st = _setup(2, 8, 8, 0.1, 1e-2, n1=beta, n3=0.0)
    u0 = _field(np.random.default_rng(32), 2, 8)
    U = O.sequential_if1(st, u0)
    u0h = np.fft.fftn(u0)
    Ep = st.E / (1.0 - st.dt * beta)
    for m in range(st.Nt):
        assert np.max(np.abs(np.fft.fftn(U[m]) - Ep ** (m + 1) * u0h)) < \
            1e-13 * np.max(np.abs(u0h))


@pytest.mark.parametrize("jac", [1, 2])
def test_if1_linear_reaction_iterates_closed_form(jac):
    """N(u) = beta u and sigma = dt beta (the mean of N' is beta): the
    preconditioned iteration is the linear one with E' = E/(1 - dt beta),
    so every iterate is (1 - psi'^k) E'^n u^_0, psi' = -alpha E'^Nt /
    (1 - alpha E'^Nt)."""
    beta, alpha = 0.8, 0.05
    st = _setup(1, 16, 8, 0.1, alpha, jac=jac, n1=beta, n3=0.0)
    u0 = _field(np.random.default_rng(33), 1, 16)
    _, _, (_, its) = O.fixed_point(st, u0, max_iter=4, tol=0.0, record=True)
    u0h = np.fft.fft(u0)
    Ep = st.E / (1.0 - st.dt * beta)
    psi = -alpha * Ep ** st.Nt / (1.0 - alpha * Ep ** st.Nt)
    for k, Uk in enumerate(its, start=1):
        for m in range(st.Nt):
            pred = (1.0 - psi ** k) * Ep ** (m + 1) * u0h
            assert np.max(np.abs(np.fft.fft(Uk[m]) - pred)) <= \
                1e-13 * np.max(np.abs(u0h))


@pytest.mark.parametrize("jac", [0, 1, 2])
@pytest.mark.parametrize("dim,n,Nt,dt", [(1, 32, 16, 0.025), (2, 16, 8, 0.05)])
def test_if1_fixed_point_reaches_sequential(jac, dim, n, Nt, dt):
    st = _setup(dim, n, Nt, dt, 1e-3, jac=jac)
    u0 = _field(np.random.default_rng(34), dim, n, amp=0.5)
    ref = O.sequential_if1(st, u0)
    U, it, _ = O.fixed_point(st, u0, tol=1e-15, max_iter=200)
    assert O.rel_err(U, ref) < 1e-13, it


def test_if1_mean_jacobian_helps():
    """With a strong reaction the averaged-Jacobian shift needs fewer
    iterations than the lagged iteration (sigma = 0)."""
    counts = []
    for jac in (0, 1):
        st = _setup(1, 32, 16, 0.05, 1e-3, jac=jac, n1=-3.0, n3=-1.0)
        u0 = _field(np.random.default_rng(35), 1, 32, amp=0.3)
        ref = O.sequential_if1(st, u0)
        _, it, _ = O.fixed_point(st, u0, ref=ref, ref_tol=1e-12,
                                 max_iter=200)
        counts.append(it)
    assert counts[1] < counts[0]


@pytest.mark.parametrize("alpha,T", [(0.2, 1.0), (0.05, 0.5), (0.3, 2.0)])
def test_if1_outer_iteration_contraction_thm_nonlin(alpha, T):
    """Theorem thm_nonlin with exact inner solves: N(u) = -u - u^3 is
    one-sided Lipschitz with M = 1 and ||e^{dt L}|| <= 1, so the error of
    every outer iteration contracts at least by
    rho = alpha q / (1 - alpha q), q = e^{-TM/(1 + 2 dt M)}."""
    Nt, n = 8, 8
    st = _setup(1, n, Nt, T / Nt, alpha, a=0.2, n1=-1.0, n3=-1.0)
    u0 = _field(np.random.default_rng(36), 1, n)
    ref = O.sequential_if1(st, u0)
    its = O.outer_iteration_if1(st, u0, 6)
    err = [np.sqrt((ref ** 2).sum(axis=1)).max()] + [
        np.sqrt(((U - ref) ** 2).sum(axis=1)).max() for U in its]
    M = 1.0
    q = math.exp(-T * M / (1.0 + 2.0 * st.dt * M))
    rho = alpha * q / (1.0 - alpha * q)
    for k in range(1, len(err)):
        if err[k - 1] < 1e-13:
            break
        assert err[k] <= rho * err[k - 1] * (1 + 1e-6) + 1e-15, (k, err)


def test_if1_printed_factor_is_too_small():
    """The factor as printed, e^{-2TM/(1 + 2 dt M)}, bounds the squared norm;
    the outer iteration's norm ratio exceeds it (so the proof's factor for
    the norm, e^{-TM/(1 + 2 dt M)}, is the one to use)."""
    alpha, T, Nt, n = 0.2, 1.0, 8, 8
    st = _setup(1, n, Nt, T / Nt, alpha, a=0.2, n1=-1.0, n3=-1.0)
    u0 = _field(np.random.default_rng(36), 1, n)
    ref = O.sequential_if1(st, u0)
    its = O.outer_iteration_if1(st, u0, 5)
    err = [np.sqrt(((U - ref) ** 2).sum(axis=1)).max() for U in its]
    q2 = math.exp(-2.0 * T / (1.0 + 2.0 * st.dt))
    printed = alpha * q2 / (1.0 - alpha * q2)
    assert max(err[k] / err[k - 1] for k in range(1, 5)) > printed
