"""GPU GMRES and Newton-GMRES vs the oracle, through the C ABI.

Results are compared, not iteration counts, except where a theorem fixes
the count (finite termination) or bounds it; GPU Arnoldi uses classical
Gram-Schmidt with delayed reorthogonalisation (DCGS2, one reduction per
step), the oracle modified Gram-Schmidt.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(
        "cuda:0")


def _solver(st, precision=0, restart=20):
    from paper_2603_04350_amd import Solver
    return Solver((st.n,) * st.dim, st.Nt, st.dt, st.alpha, st.scheme,
                  st.a, st.c, st.n1, st.n2, st.n3, precision, restart)


def _zeros(st):
    import torch
    return torch.zeros((st.Nt,) + (st.n,) * st.dim, dtype=torch.float64,
                       device="cuda:0")


LINEAR = {
    "heat1d_C1": (1, 64, 16, 1e-2, 1.0, 0.0),
    "heat2d": (2, 32, 32, 1e-3, 0.1, 0.1),
    "heat3d": (3, 16, 8, 1e-2, 1.0, 0.0),
    "heat1d_alpha02": (1, 32, 64, 0.2, 0.05, 0.0),
}


@pytest.mark.parametrize("case", sorted(LINEAR))
def test_linear_gmres_solution(case):
    dim, n, Nt, alpha, a, c = LINEAR[case]
    st = O.Setup(dim, n, Nt, 1.0 / Nt, alpha, a, c)
    rng = np.random.default_rng([n, Nt])
    u0 = rng.uniform(-0.9, 0.9, size=(n,) * dim)
    ref = O.sequential(st, u0)
    Uo, it_o, _ = O.gmres_solve(st, u0, restart=20, tol=1e-13)
    with _solver(st) as s:
        U = _zeros(st)
        rc, it, rel = s.gmres(_dev(u0), U, restart=20, max_iter=200,
                              tol=1e-13)
    assert rel <= 1e-13
    assert O.rel_err(U.cpu().numpy(), ref) < 1e-12
    assert abs(it - it_o) <= 1, (it, it_o)


def test_gmres_residual_bound_gmres3_thm():
    """||r_k|| <= (4 alpha (1 - alpha))^{k/2} ||r_0||: after k iterations
    the GPU's relative preconditioned residual respects the bound."""
    import math
    st = O.Setup(1, 32, 8, 0.1, 0.1, a=0.3)
    u0 = np.random.default_rng(3).uniform(-0.9, 0.9, size=32)
    with _solver(st) as s:
        for k in (1, 2, 3):
            U = _zeros(st)
            rc, it, rel = s.gmres(_dev(u0), U, restart=k, max_iter=k,
                                  tol=1e-15)
            assert rel <= math.sqrt(4 * 0.1 * 0.9) ** k * (1 + 1e-8)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_newton_gmres_reaches_sequential(scheme, precision):
    inst = W.scaled(W.rd2d(), n=32, Nt=32)
    inst.scheme = scheme
    st = O.Setup.from_instance(inst)
    ref = O.sequential(st, inst.u0)
    with _solver(st, precision=precision) as s:
        U = _zeros(st)
        rc, it, rel = s.gmres(_dev(inst.u0), U, restart=20, max_iter=400,
                              tol=1e-12)
    err = O.rel_err(U.cpu().numpy(), ref)
    assert err < 1e-10, (it, rel, err)
    assert it // 1000 <= 12


def test_newton_gmres_3d_and_1d():
    for dim, n in ((1, 64), (3, 16)):
        st = O.Setup(dim, n, 16, 1.0 / 16, 1e-3, a=0.05, n1=1.0, n3=-1.0,
                     scheme=2)
        u0 = np.random.default_rng(dim).uniform(-0.9, 0.9, size=(n,) * dim)
        ref = O.sequential(st, u0)
        with _solver(st) as s:
            U = _zeros(st)
            rc, it, rel = s.gmres(_dev(u0), U, restart=20, max_iter=400,
                                  tol=1e-12)
        assert O.rel_err(U.cpu().numpy(), ref) < 1e-10


JVP_CASES = {
    # (dim, n, Nt, scheme, precision): 1D/2D/3D, ETD1/ETD2, fp64 and the
    # fp32 Jacobian products of mixed precision (d >= 2), a 2D grid whose
    # columns span several tiles, and a non-square time/space ratio
    "1d_etd1": (1, 64, 16, 1, 0),
    "1d_etd2": (1, 128, 8, 2, 0),
    "2d_etd1": (2, 32, 16, 1, 0),
    "2d_etd2": (2, 64, 32, 2, 0),
    "2d_etd2_n256": (2, 256, 8, 2, 0),
    "3d_etd2": (3, 16, 8, 2, 0),
    "2d_etd1_mixed": (2, 32, 16, 1, 1),
    "2d_etd2_mixed": (2, 64, 32, 2, 1),
    "3d_etd2_mixed": (3, 16, 8, 2, 1),
}


@pytest.mark.parametrize("case", sorted(JVP_CASES))
def test_newton_operator_parity(case):
    """The device's Newton operator Q_alpha^{-1}(Q - G'(U)) V (Sec. 5, eq.
    newton_2 on the all-at-once system) element by element against the
    oracle's q_apply, gprime_apply and precond_apply on the same seeded U,
    V (Allen-Cahn reaction N = u - u^3, so N' = 1 - 3u^2 varies in space
    and time).  fp64: 1e-12 of the largest entry; mixed (fp32 products
    N'(u) v and their FFTs): 1e-5, the per-application bar of mixed mode.
    A second call at a different U on the same handle checks that no state
    of the first survives."""
    dim, n, Nt, scheme, precision = JVP_CASES[case]
    st = O.Setup(dim, n, Nt, 1.0 / Nt, 1e-2, a=0.05, n1=1.0, n3=-1.0,
                 scheme=scheme)
    rng = np.random.default_rng([dim, n, Nt, scheme])
    u0 = rng.uniform(-0.9, 0.9, size=(n,) * dim)
    bar = 1e-12 if precision == 0 else 1e-5
    import torch
    with _solver(st, precision=precision, restart=2) as s:
        for trial in range(2):
            U = rng.uniform(-1.0, 1.0, size=(Nt,) + (n,) * dim)
            V = rng.standard_normal((Nt,) + (n,) * dim)
            ref = O.precond_apply(st, O.q_apply(st, V)
                                  - O.gprime_apply(st, u0, U, V))
            Wd = torch.empty_like(_dev(V))
            s.newton_apply(_dev(u0), _dev(U), _dev(V), Wd)
            got = Wd.cpu().numpy()
            err = np.abs(got - ref).max() / np.abs(ref).max()
            assert err < bar, (case, trial, err)
            # the Jacobian term is not negligible in the operator
            lin = O.precond_apply(st, O.q_apply(st, V))
            assert np.abs(lin - ref).max() > 1e3 * bar * np.abs(ref).max()


def test_newton_operator_linear_is_gmres_operator():
    """Linear problems: W = Q_alpha^{-1} Q V (the GMRES operator of Sec.
    3.2), element by element."""
    import torch
    st = O.Setup(2, 32, 16, 1.0 / 16, 1e-2, a=0.1)
    rng = np.random.default_rng(11)
    u0 = rng.uniform(-0.9, 0.9, size=(32, 32))
    V = rng.standard_normal((16, 32, 32))
    ref = O.precond_apply(st, O.q_apply(st, V))
    with _solver(st, restart=1) as s:
        Wd = torch.empty_like(_dev(V))
        s.newton_apply(_dev(u0), _dev(np.zeros_like(V)), _dev(V), Wd)
    err = np.abs(Wd.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err


def test_rd2d_full_size_newton_gmres():
    """The reaction-diffusion configuration at full size: 512^2 x 128, ETD2,
    Exp-ParaDiag as the GMRES(20) preconditioner to tol 1e-10, mixed
    precision (fp32 Jacobian products, fp64 residual and time
    diagonalisation).  The window is held against sequential ETD2 stepping
    in fp64 at the mixed-mode bar 1e-10.  Newton stops on the residual,
    ||R_j|| <= tol ||R_0||, and the error is about the residual's size (a
    stop at 1e-10 can land just above the bar), so the solve runs to tol
    1e-11."""
    import torch
    from paper_2603_04350_amd import Solver
    inst = W.rd2d()
    st = O.Setup.from_instance(inst)
    ref = O.sequential(st, inst.u0)
    with Solver.from_instance(inst, gmres_restart=20) as s:
        U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64,
                        device="cuda:0")
        rc, it, rel = s.gmres(_dev(inst.u0), U, restart=20, max_iter=400,
                              tol=1e-11)
    assert rc == 0 and rel <= 1e-11
    err = O.rel_err(U.cpu().numpy(), ref)
    print(f"rd2d 512^2 x 128 Newton-GMRES: {it // 1000} Newton steps, "
          f"{it % 1000} GMRES iterations, error {err:.2e}")
    assert err < 1e-10, (it, rel, err)
