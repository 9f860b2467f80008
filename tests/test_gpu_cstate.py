"""GPU library with a complex state (the Schroedinger equation of Sec. 6,
a = i) vs the CPU oracle, through the C ABI.

Physical arrays are complex128 (interleaved), the spectral state is the full
spectrum, the symbol is complex and not Hermitian.  Tolerances as in
test_gpu_parity: residual 1e-13 relative, preconditioner and iterates
max(1e-12, 50 eps/alpha), converged windows 1e-12 against sequential
stepping.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

EPS = 2.220446049250313e-16

# (dim, n, Nt, alpha, a, a_im, c, c_im, scheme)
CASES = {
    "se1d": (1, 64, 16, 1e-2, 0.0, 1.0, 0.0, 2.0, 1),
    "se1d_n4_Nt2": (1, 4, 2, 0.3, 0.0, 1.0, 0.0, 2.0, 1),
    "se2d": (2, 16, 32, 1e-3, 0.0, 1.0, 0.0, 200.0, 1),
    "se2d_rect_damped": (2, 8, 64, 1e-3, 0.05, 1.0, 0.1, 2.0, 1),
    "se3d": (3, 8, 8, 1e-2, 0.0, 1.0, 0.0, 2.0, 1),
    "se1d_last1024": (1, 1024, 4, 1e-2, 0.0, 1e-4, 0.0, 0.0, 1),
    "se2d_ebdf2_fft": (2, 16, 17, 1e-3, 0.0, 1.0, 0.0, 2.0, 3),
    "se1d_ebdf2_dense": (1, 32, 16, 1e-2, 0.0, 1.0, 0.0, 2.0, 3),
}


def _setup(case, T=1.0):
    dim, n, Nt, alpha, a, a_im, c, c_im, scheme = CASES[case]
    return O.Setup(dim, n, Nt, T / Nt, alpha, a, c, scheme=scheme,
                   a_im=a_im, c_im=c_im)


def _u0(st, seed=0):
    rng = np.random.default_rng([seed, st.n, st.Nt, 17])
    sh = (st.n,) * st.dim
    return rng.uniform(-0.9, 0.9, size=sh) + 1j * rng.uniform(-0.9, 0.9,
                                                               size=sh)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _zeros(st):
    import torch
    return torch.zeros((st.Nt,) + (st.n,) * st.dim, dtype=torch.complex128,
                       device="cuda:0")


def _solver(st, restart=0):
    from paper_2603_04350_amd import Solver
    return Solver((st.n,) * st.dim, st.Nt, st.dt, st.alpha, st.scheme,
                  st.a, st.c, 0.0, 0.0, 0.0, 0, restart, a_im=st.a_im,
                  c_im=st.c_im, complex_state=1)


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
def test_cstate_residual_parity(case):
    import torch
    st = _setup(case)
    u0 = _u0(st)
    rng = np.random.default_rng(1)
    sh = (st.Nt,) + (st.n,) * st.dim
    U = 0.5 * (rng.standard_normal(sh) + 1j * rng.standard_normal(sh))
    with _solver(st) as s:
        R = torch.empty_like(_dev(U))
        rn = s.residual(_dev(u0), _dev(U), R)
        torch.cuda.synchronize()
    Rr = _residual(st, u0, U)
    assert _rel(R.cpu().numpy(), Rr) < 1e-13
    assert abs(rn - np.linalg.norm(Rr)) < 1e-12 * np.linalg.norm(Rr)


@pytest.mark.parametrize("case", sorted(CASES))
def test_cstate_precond_parity(case):
    import torch
    st = _setup(case)
    rng = np.random.default_rng(2)
    sh = (st.Nt,) + (st.n,) * st.dim
    Rv = rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
    with _solver(st) as s:
        S = torch.empty_like(_dev(Rv))
        s.precond_apply(_dev(Rv), S)
        torch.cuda.synchronize()
    assert _rel(S.cpu().numpy(), _precond(st, Rv)) < _bar(st)


@pytest.mark.parametrize("case", sorted(CASES))
def test_cstate_iterates_parity(case):
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
def test_cstate_converged_equals_sequential(case):
    st = _setup(case)
    u0 = _u0(st)
    ref = O.sequential(st, u0)
    with _solver(st) as s:
        U = _zeros(st)
        rc, it, rel = s.iterate(_dev(u0), U, max_iter=400, tol=1e-14)
    err = O.rel_err(U.cpu().numpy(), ref)
    assert err < 1e-12, (it, rel, err)


def test_schroedinger_plane_waves_and_norm_on_gpu():
    """e^{3ix} + 0.5 e^{-2ix} under u_t = i u_xx - 2i u: exact rotation of
    each wave, and the l2 norm of every slice equals that of u_0."""
    n, Nt, T = 64, 32, 1.0
    st = O.Setup(1, n, Nt, T / Nt, 1e-3, a=0.0, a_im=1.0, c_im=2.0)
    x = 2 * np.pi * np.arange(n) / n
    u0 = np.exp(3j * x) + 0.5 * np.exp(-2j * x)
    t = (np.arange(Nt) + 1) * T / Nt
    ex = np.array([np.exp(-11j * tt) * np.exp(3j * x)
                   + 0.5 * np.exp(-6j * tt) * np.exp(-2j * x) for tt in t])
    with _solver(st) as s:
        U = _zeros(st)
        s.iterate(_dev(u0), U, max_iter=100, tol=1e-14)
    Ug = U.cpu().numpy()
    assert np.max(np.abs(Ug - ex)) < 1e-13
    nrm = np.linalg.norm(u0)
    assert np.max(np.abs(np.linalg.norm(Ug, axis=1) - nrm)) < 1e-13 * nrm


@pytest.mark.parametrize("case", ["se1d", "se2d", "se3d", "se2d_ebdf2_fft"])
def test_cstate_gmres(case):
    st = _setup(case)
    u0 = _u0(st)
    ref = O.sequential(st, u0)
    with _solver(st, restart=20) as s:
        U = _zeros(st)
        rc, it, rel = s.gmres(_dev(u0), U, restart=20, max_iter=200,
                              tol=1e-13)
    assert rel <= 1e-13
    assert O.rel_err(U.cpu().numpy(), ref) < 1e-12
    # complex GMRES (one complex dimension per step) needs no more steps
    # than GMRES on the real form of the system, the oracle's
    solve = O.gmres_solve_ebdf2 if st.scheme == O.EBDF2 else O.gmres_solve
    _, it_real, _ = solve(st, u0, restart=20, tol=1e-13)
    assert it <= it_real, (it, it_real)


def test_cstate_heat_with_complex_data():
    """A real operator on a complex state: real and imaginary parts evolve
    as two independent real heat solutions."""
    st = O.Setup(2, 16, 16, 1.0 / 16, 1e-2, a=0.3, c=0.1, cstate=True)
    rng = np.random.default_rng(4)
    ur = rng.uniform(-0.9, 0.9, (16, 16))
    ui = rng.uniform(-0.9, 0.9, (16, 16))
    str_ = O.Setup(2, 16, 16, 1.0 / 16, 1e-2, a=0.3, c=0.1)
    ref = O.sequential(str_, ur) + 1j * O.sequential(str_, ui)
    from paper_2603_04350_amd import Solver
    with Solver((16, 16), 16, 1.0 / 16, 1e-2, 1, 0.3, 0.1,
                complex_state=1) as s:
        U = _zeros(st)
        s.iterate(_dev(ur + 1j * ui), U, max_iter=100, tol=1e-14)
    assert O.rel_err(U.cpu().numpy(), ref) < 1e-12


def test_cstate_in_batch_with_real_instances():
    """A batch holding complex-state and real-state instances: each result
    is bitwise the one its handle gives alone."""
    import torch
    from paper_2603_04350_amd import Batch, Solver
    sts = [_setup("se2d"), _setup("se1d"), _setup("se2d_ebdf2_fft")]
    solvers = [_solver(st) for st in sts]
    u0s = [_u0(st) for st in sts]
    rs = O.Setup(2, 32, 16, 1.0 / 16, 1e-3, a=0.0025, n1=1.0, n3=-1.0)
    solvers.append(Solver((32, 32), 16, rs.dt, rs.alpha, 1, rs.a, 0.0, 1.0,
                          0.0, -1.0))
    u0r = np.random.default_rng(3).uniform(-0.9, 0.9, (32, 32))
    tens = [_dev(u) for u in u0s] + [_dev(u0r)]
    shapes = [((st.Nt,) + (st.n,) * st.dim, torch.complex128) for st in sts]
    shapes.append(((16, 32, 32), torch.float64))
    solo = []
    for s, t, (sh, dt) in zip(solvers, tens, shapes):
        U = torch.zeros(sh, dtype=dt, device="cuda:0")
        s.iterate(t, U, max_iter=200, tol=1e-12)
        solo.append(U.cpu().numpy())
    b = Batch(solvers)
    Us = [torch.zeros(sh, dtype=dt, device="cuda:0") for sh, dt in shapes]
    b.iterate(tens, Us, max_iter=200, tol=1e-12)
    b.close()
    for k in range(len(Us)):
        assert np.array_equal(Us[k].cpu().numpy(), solo[k]), k
    for s in solvers:
        s.close()


def test_schroedinger_full_size_2d_256():
    """The Schroedinger benchmark instance (256^2 x 64, wave packet):
    converged window against sequential stepping."""
    inst = W.schroedinger2d()
    st = O.Setup.from_instance(inst)
    ref = O.sequential(st, inst.u0)
    from paper_2603_04350_amd import Solver
    with Solver.from_instance(inst) as s:
        U = _zeros(st)
        rc, it, rel = s.iterate(_dev(inst.u0), U, max_iter=100, tol=1e-11)
    assert rc == 0
    assert O.rel_err(U.cpu().numpy(), ref) < 1e-10, (it, rel)


def test_cstate_argument_errors():
    from paper_2603_04350_amd import expdiag as X
    with pytest.raises(RuntimeError):   # complex coefficients, real state
        X.Solver((16,), 8, 0.1, 1e-2, 1, 0.0, a_im=1.0, complex_state=0)
    with pytest.raises(RuntimeError):   # complex state is linear only
        X.Solver((16,), 8, 0.1, 1e-2, 1, 0.1, n1=1.0, complex_state=1)
