"""GPU library with complex symbols (periodic advection-diffusion, the remark
after Theorem thm_gmres22) vs the CPU oracle, through the C ABI.

E_k = e^{dt mu_k} with mu_k = -a|k|^2 - c - i b.k' is complex; the state
stays real (Hermitian symbol), so the half spectrum carries it exactly.
Tolerances as in test_gpu_parity: residual 1e-13 relative, preconditioner
and iterates max(1e-12, 50 eps/alpha), converged results 1e-12 against
sequential stepping.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

EPS = 2.220446049250313e-16

# (dim, n, Nt, alpha, a, c, n1, n3, scheme, b)
CASES = {
    "ade1d": (1, 64, 16, 1e-2, 0.1, 0.0, 0, 0, 1, (2.0, 0, 0)),
    "ade1d_adv_dominated": (1, 128, 32, 1e-3, 1e-5, 0.0, 0, 0, 1, (2.0, 0, 0)),
    "ade2d_ragged": (2, 8, 64, 1e-3, 0.05, 0.1, 0, 0, 1, (1.0, -0.5, 0)),
    "ade3d": (3, 8, 8, 1e-2, 0.3, 0.0, 0, 0, 1, (0.5, 1.0, -1.5)),
    "ac_adv2d_etd1": (2, 32, 16, 1e-3, 0.0025, 0.0, 1.0, -1.0, 1, (2.0, 1.0, 0)),
    "ac_adv1d_etd2": (1, 32, 32, 1e-3, 0.01, 0.0, 1.0, -1.0, 2, (1.5, 0, 0)),
    "ade2d_ebdf2_fft": (2, 16, 17, 1e-3, 0.05, 0.0, 0, 0, 3, (2.0, 1.0, 0)),
    "ade1d_ebdf2_dense": (1, 64, 16, 1e-2, 0.1, 0.0, 0, 0, 3, (2.0, 0, 0)),
}


def _setup(case, T=1.0):
    dim, n, Nt, alpha, a, c, n1, n3, scheme, b = CASES[case]
    return O.Setup(dim, n, Nt, T / Nt, alpha, a, c, n1, 0.0, n3, scheme,
                   tuple(float(v) for v in b))


def _u0(st, seed=0):
    rng = np.random.default_rng([seed, st.n, st.Nt, 11])
    return rng.uniform(-0.9, 0.9, size=(st.n,) * st.dim)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(
        "cuda:0")


def _zeros(st):
    import torch
    return torch.zeros((st.Nt,) + (st.n,) * st.dim, dtype=torch.float64,
                       device="cuda:0")


def _solver(st, restart=0):
    from paper_2603_04350_amd import Solver
    return Solver((st.n,) * st.dim, st.Nt, st.dt, st.alpha, st.scheme,
                  st.a, st.c, st.n1, st.n2, st.n3, 0, restart, b=st.b)


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _bar(st):
    return max(1e-12, 50 * EPS / st.alpha)


def _residual(st, u0, U):
    if st.scheme == O.EBDF2:
        return O.residual_ebdf2(st, u0, U)
    return O.residual(st, u0, U)


def _precond(st, R):
    if st.scheme == O.EBDF2:
        return O.precond_apply_ebdf2(st, R)
    return O.precond_apply(st, R)


@pytest.mark.parametrize("case", sorted(CASES))
def test_complex_symbol_residual_parity(case):
    import torch
    st = _setup(case)
    u0 = _u0(st)
    U = 0.5 * np.random.default_rng(1).standard_normal(
        (st.Nt,) + (st.n,) * st.dim)
    with _solver(st) as s:
        R = torch.empty_like(_dev(U))
        s.residual(_dev(u0), _dev(U), R)
        torch.cuda.synchronize()
    assert _rel(R.cpu().numpy(), _residual(st, u0, U)) < 1e-13


@pytest.mark.parametrize("case", sorted(CASES))
def test_complex_symbol_precond_parity(case):
    import torch
    st = _setup(case)
    Rv = np.random.default_rng(2).standard_normal((st.Nt,) + (st.n,) * st.dim)
    with _solver(st) as s:
        S = torch.empty_like(_dev(Rv))
        s.precond_apply(_dev(Rv), S)
        torch.cuda.synchronize()
    assert _rel(S.cpu().numpy(), _precond(st, Rv)) < _bar(st)


@pytest.mark.parametrize("case", sorted(CASES))
def test_complex_symbol_iterates_parity(case):
    st = _setup(case)
    u0 = _u0(st)
    _, _, (_, its) = O.fixed_point(st, u0, max_iter=3, tol=0.0, record=True)
    with _solver(st) as s:
        for k in (1, 2, 3):
            U = _zeros(st)
            rc, it, rel = s.iterate(_dev(u0), U, max_iter=k, tol=0.0)
            assert it == k
            err = O.rel_err(U.cpu().numpy(), its[k - 1])
            assert err < _bar(st), (k, err)


@pytest.mark.parametrize("case", sorted(CASES))
def test_complex_symbol_converged_equals_sequential(case):
    st = _setup(case)
    u0 = _u0(st)
    ref = O.sequential(st, u0)
    with _solver(st) as s:
        U = _zeros(st)
        rc, it, rel = s.iterate(_dev(u0), U, max_iter=400, tol=1e-14)
    err = O.rel_err(U.cpu().numpy(), ref)
    assert err < 1e-12, (it, rel, err)


def test_advection_exact_solution_on_gpu():
    """u_t = a u_xx - b u_x from trigonometric data: the GPU window equals
    the advected, damped modes (exact in time for the linear problem)."""
    n, Nt, T, a, b = 64, 32, 1.0, 0.1, 2.0
    st = O.Setup(1, n, Nt, T / Nt, 1e-3, a=a, b=(b, 0.0, 0.0))
    x = 2 * np.pi * np.arange(n) / n
    u0 = np.sin(x) + 0.3 * np.cos(3 * x)
    t = (np.arange(Nt) + 1) * T / Nt
    ex = np.array([np.exp(-a * tt) * np.sin(x - b * tt)
                   + 0.3 * np.exp(-9 * a * tt) * np.cos(3 * (x - b * tt))
                   for tt in t])
    with _solver(st) as s:
        U = _zeros(st)
        s.iterate(_dev(u0), U, max_iter=100, tol=1e-14)
    assert np.max(np.abs(U.cpu().numpy() - ex)) < 1e-13


@pytest.mark.parametrize("case", ["ade1d", "ade2d_ragged", "ade3d",
                                  "ade2d_ebdf2_fft"])
def test_complex_symbol_gmres(case):
    st = _setup(case)
    u0 = _u0(st)
    ref = O.sequential(st, u0)
    with _solver(st, restart=20) as s:
        U = _zeros(st)
        rc, it, rel = s.gmres(_dev(u0), U, restart=20, max_iter=200,
                              tol=1e-13)
    assert rel <= 1e-13
    assert O.rel_err(U.cpu().numpy(), ref) < 1e-12


def test_advection_newton_gmres():
    st = _setup("ac_adv2d_etd1")
    u0 = _u0(st)
    with _solver(st, restart=20) as s:
        U = _zeros(st)
        rc, it, rel = s.gmres(_dev(u0), U, restart=20, max_iter=400,
                              tol=1e-11)
    assert O.rel_err(U.cpu().numpy(), O.sequential(st, u0)) < 1e-10


def test_advection_full_size_2d_256():
    """The advection benchmark instance (Allen-Cahn 256^2 x 64 with
    b = (2, 1)): converged window against sequential stepping."""
    import workloads as W
    inst = W.advection2d()
    st = O.Setup.from_instance(inst)
    ref = O.sequential(st, inst.u0)
    from paper_2603_04350_amd import Solver
    with Solver.from_instance(inst) as s:
        U = _zeros(st)
        rc, it, rel = s.iterate(_dev(inst.u0), U, max_iter=200, tol=1e-11)
    assert rc == 0
    assert O.rel_err(U.cpu().numpy(), ref) < 1e-10, (it, rel)
