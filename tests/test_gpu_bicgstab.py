"""GPU preconditioned BiCGStab and Newton-BiCGStab vs the oracle, through
the C ABI.

The first iterates are compared element by element with the oracle's
BiCGStab on the same left-preconditioned system (same shadow residual, same
order of updates): after k iterations both hold the same Krylov-space
combination, so the iterates differ by the rounding of k operator
applications and inner products, amplified by the conditioning of the
alpha-scaled diagonalisation; the bar is max(1e-11, 500 eps / alpha)
relative.  Converged solutions are held to 1e-12 against sequential
stepping, iteration counts to the oracle's within one.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

EPS = 2.220446049250313e-16

# (scheme, dim, n, Nt, alpha, a, c)
LINEAR = {
    "etd1_heat1d": (1, 1, 64, 16, 1e-2, 1.0, 0.0),
    "etd1_heat2d": (1, 2, 32, 32, 1e-3, 0.1, 0.1),
    "etd1_heat3d_ragged": (1, 3, 8, 8, 1e-2, 1.0, 0.0),
    "etd1_heat1d_alpha02": (1, 1, 32, 64, 0.2, 0.05, 0.0),
    "ebdf2_fft_heat2d": (O.EBDF2, 2, 16, 17, 1e-3, 0.3, 0.0),
    "ebdf2_dense_heat1d": (O.EBDF2, 1, 64, 32, 1e-2, 0.2, 0.0),
    "ebdf4_fft_heat1d": (O.EBDF4, 1, 64, 19, 1e-2, 0.1, 0.0),
    "ebdf6_dense_heat2d": (O.EBDF6, 2, 16, 16, 1e-3, 0.05, 0.0),
}


def _setup(case):
    scheme, dim, n, Nt, alpha, a, c = LINEAR[case]
    return O.Setup(dim, n, Nt, 1.0 / Nt, alpha, a, c, scheme=scheme)


def _u0(st, seed=0):
    rng = np.random.default_rng([seed, st.n, st.Nt, 13])
    return rng.uniform(-0.9, 0.9, size=(st.n,) * st.dim)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _zeros(st, dtype=None):
    import torch
    return torch.zeros((st.Nt,) + (st.n,) * st.dim,
                       dtype=dtype or torch.float64, device="cuda:0")


def _solver(st, restart=8, precision=0):
    from paper_2603_04350_amd import Solver
    return Solver((st.n,) * st.dim, st.Nt, st.dt, st.alpha, st.scheme,
                  st.a, st.c, st.n1, st.n2, st.n3, precision, restart)


@pytest.mark.parametrize("case", sorted(LINEAR))
def test_bicgstab_iterates_parity(case):
    st = _setup(case)
    u0 = _u0(st)
    bar = max(1e-11, 500 * EPS / st.alpha)
    with _solver(st) as s:
        for k in (1, 2, 3):
            Uo, it_o, _ = O.bicgstab_solve(st, u0, tol=0.0, max_iter=k)
            assert it_o == k
            U = _zeros(st)
            rc, it, rel = s.bicgstab(_dev(u0), U, max_iter=k, tol=1e-300)
            assert it == k
            assert O.rel_err(U.cpu().numpy(), Uo) < bar, k


@pytest.mark.parametrize("case", sorted(LINEAR))
def test_bicgstab_solution(case):
    st = _setup(case)
    u0 = _u0(st)
    ref = O.sequential(st, u0)
    _, it_o, _ = O.bicgstab_solve(st, u0, tol=1e-13)
    with _solver(st) as s:
        U = _zeros(st)
        rc, it, rel = s.bicgstab(_dev(u0), U, max_iter=200, tol=1e-13)
    assert rc == 0 and rel <= 1e-13
    assert O.rel_err(U.cpu().numpy(), ref) < 1e-12
    assert abs(it - it_o) <= 1, (it, it_o)


def test_bicgstab_complex_state():
    st = O.Setup(2, 16, 32, 1.0 / 32, 1e-3, a=0.0, a_im=1.0, c_im=200.0)
    rng = np.random.default_rng(4)
    u0 = rng.uniform(-1, 1, (16, 16)) + 1j * rng.uniform(-1, 1, (16, 16))
    import torch
    from paper_2603_04350_amd import Solver
    with Solver((16, 16), 32, st.dt, st.alpha, 1, 0.0, 0.0, 0.0, 0.0, 0.0,
                0, 8, a_im=1.0, c_im=200.0, complex_state=1) as s:
        U = _zeros(st, torch.complex128)
        rc, it, rel = s.bicgstab(_dev(u0), U, max_iter=100, tol=1e-13)
    assert rel <= 1e-13
    assert O.rel_err(U.cpu().numpy(), O.sequential(st, u0)) < 1e-12
    _, it_o, _ = O.bicgstab_solve(st, u0, tol=1e-13)
    assert abs(it - it_o) <= 1, (it, it_o)


def test_bicgstab_no_more_operator_work_than_gmres():
    """On the heat problem of Table cpu_time_combined's kind (alpha small,
    spectrum clustered at one) BiCGStab reaches the tolerance within the
    operator applications GMRES needs, or one more iteration's worth."""
    st = _setup("etd1_heat2d")
    u0 = _u0(st)
    with _solver(st, restart=20) as s:
        U = _zeros(st)
        _, it_b, _ = s.bicgstab(_dev(u0), U, max_iter=100, tol=1e-12)
        U = _zeros(st)
        _, it_g, _ = s.gmres(_dev(u0), U, restart=20, max_iter=100,
                             tol=1e-12)
    assert 2 * it_b <= it_g + 2, (it_b, it_g)


@pytest.mark.parametrize("scheme,precision", [(1, 0), (2, 0), (1, 1)])
def test_newton_bicgstab_reaches_sequential(scheme, precision):
    st = O.Setup(2, 32, 16, 1.0 / 16, 1e-3, a=0.0025, n1=1.0, n3=-1.0,
                 scheme=scheme)
    u0 = np.random.default_rng(5).uniform(-0.9, 0.9, (32, 32))
    ref = O.sequential(st, u0)
    with _solver(st, precision=precision) as s:
        U = _zeros(st)
        rc, it, rel = s.bicgstab(_dev(u0), U, max_iter=400, tol=1e-11)
    assert rc == 0
    assert O.rel_err(U.cpu().numpy(), ref) < (1e-10 if precision else 1e-11)


def test_newton_bicgstab_matches_oracle_newton():
    """Same Newton outer loop and forcing term as the oracle's
    newton_bicgstab: the same number of Newton steps and the same window."""
    st = O.Setup(1, 64, 16, 1.0 / 16, 1e-2, a=0.01, n1=1.0, n3=-1.0)
    u0 = np.random.default_rng(6).uniform(-0.9, 0.9, 64)
    Uo, newton_o, _, _ = O.newton_bicgstab(st, u0, tol=1e-11)
    with _solver(st) as s:
        U = _zeros(st)
        rc, it, rel = s.bicgstab(_dev(u0), U, max_iter=400, tol=1e-11)
    assert it // 1000 == newton_o, (it, newton_o)
    assert O.rel_err(U.cpu().numpy(), Uo) < 1e-11


def test_if1_newton_bicgstab():
    st = O.Setup(1, 64, 16, 0.025, 1e-3, a=0.01, n1=1.0, n3=-1.0,
                 scheme=O.IF1)
    u0 = np.random.default_rng(7).uniform(-0.9, 0.9, 64)
    from paper_2603_04350_amd import Solver
    with Solver((64,), 16, st.dt, st.alpha, O.IF1, st.a, 0.0, 1.0, 0.0,
                -1.0, 0, 8) as s:
        U = _zeros(st)
        rc, it, rel = s.bicgstab(_dev(u0), U, max_iter=400, tol=1e-12)
    assert O.rel_err(U.cpu().numpy(), O.sequential_if1(st, u0)) < 1e-11


def test_bicgstab_argument_errors():
    from paper_2603_04350_amd import Solver
    st = _setup("etd1_heat1d")
    with _solver(st, restart=4) as s:          # workspace too small
        with pytest.raises(RuntimeError):
            s.bicgstab(_dev(_u0(st)), _zeros(st), max_iter=10, tol=1e-10)
    with _solver(st) as s:
        with pytest.raises(RuntimeError):
            s.bicgstab(_dev(_u0(st)), _zeros(st), max_iter=0, tol=1e-10)
        with pytest.raises(RuntimeError):
            s.bicgstab(_dev(_u0(st)), _zeros(st), max_iter=10, tol=0.0)
