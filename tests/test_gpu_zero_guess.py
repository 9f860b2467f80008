"""Solves from the all-zero initial iterate (expdiag_set_zero_guess,
expdiag_batch_set_zero_guess) against the same solves from a zeroed U,
through the C ABI.

With the option the library clears the spectral iterate (and the fp32 bulk
copy of a mixed instance) instead of transforming U, and never reads U: the
results must equal those of a solve from a zeroed U bit for bit, also when
U holds NaN on entry.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _full(shape, value, dtype=None):
    import torch
    return torch.full(shape, value, dtype=dtype or torch.float64,
                      device="cuda:0")


def _shape(inst):
    return (inst.Nt,) + inst.shape


# name -> (instance, precision)
SINGLE = {
    "ac2d_fp64": (W.scaled(W.allen_cahn2d(), 32, 16), 0),
    "ac2d_mixed_bulk_fp32": (W.scaled(W.allen_cahn2d(), 64, 16), 1),
    "rd2d_etd2_mixed": (W.scaled(W.rd2d(), 32, 16), 1),
    "heat1d": (W.heat1d(), 0),
    "ebdf2_dense_Nt16": (W.diffusion2d_ebdf(2, n=32, Nt=16), 0),
    "ebdf4_fft_Nt19": (W.diffusion2d_ebdf(4, n=32, Nt=19), 0),
}


@pytest.mark.parametrize("case", sorted(SINGLE))
def test_fixed_point_from_zero_guess_equals_zeroed_U(case):
    from paper_2603_04350_amd import Solver
    inst, prec = SINGLE[case]
    u0 = _dev(inst.u0)
    with Solver.from_instance(inst, precision=prec) as s:
        U = _full(_shape(inst), 0.0)
        rc, it, rel = s.iterate(u0, U, max_iter=200, tol=1e-12)
        ref = U.cpu().numpy()
        s.set_zero_guess(True)
        for _ in range(2):  # the second solve starts from the first's count
            U = _full(_shape(inst), float("nan"))
            rc2, it2, rel2 = s.iterate(u0, U, max_iter=200, tol=1e-12)
            assert it2 == it and rel2 == rel
            assert np.array_equal(U.cpu().numpy(), ref)
        s.set_zero_guess(False)
        U = _full(_shape(inst), 0.0)
        s.iterate(u0, U, max_iter=200, tol=1e-12)
        assert np.array_equal(U.cpu().numpy(), ref)


@pytest.mark.parametrize("method", ["gmres", "bicgstab"])
@pytest.mark.parametrize("case", ["heat1d", "ebdf2_dense_Nt16"])
def test_krylov_from_zero_guess_equals_zeroed_U(case, method):
    from paper_2603_04350_amd import Solver
    inst, prec = SINGLE[case]
    u0 = _dev(inst.u0)
    with Solver.from_instance(inst, gmres_restart=20, precision=prec) as s:
        solve = s.gmres if method == "gmres" else s.bicgstab
        U = _full(_shape(inst), 0.0)
        out = solve(u0, U, max_iter=100, tol=1e-10)
        ref = U.cpu().numpy()
        s.set_zero_guess(True)
        U = _full(_shape(inst), float("nan"))
        assert solve(u0, U, max_iter=100, tol=1e-10) == out
        assert np.array_equal(U.cpu().numpy(), ref)


def _cstate_solver():
    from paper_2603_04350_amd import Solver
    n, Nt, alpha = 16, 32, 1e-3
    return Solver((n, n), Nt, 1.0 / Nt, alpha, 1, 0.0, 0.0, 0.0, 0.0, 0.0,
                  0, 0, a_im=1.0, c_im=200.0, complex_state=1), (Nt, n, n)


def _cstate_u0():
    rng = np.random.default_rng(7)
    return (rng.uniform(-0.9, 0.9, (16, 16)) +
            1j * rng.uniform(-0.9, 0.9, (16, 16)))


def test_complex_state_from_zero_guess_equals_zeroed_U():
    import torch
    s, sh = _cstate_solver()
    u0 = _dev(_cstate_u0())
    U = _full(sh, 0.0, torch.complex128)
    rc, it, rel = s.iterate(u0, U, max_iter=200, tol=1e-12)
    ref = U.cpu().numpy()
    s.set_zero_guess(True)
    U = _full(sh, complex(float("nan"), float("nan")), torch.complex128)
    assert s.iterate(u0, U, max_iter=200, tol=1e-12)[1] == it
    assert np.array_equal(U.cpu().numpy(), ref)
    s.close()


def test_batch_from_zero_guess_equals_zeroed_Us():
    """Real instances of both precisions and shapes (entry plan: the cleared
    iterates as one job-table launch) and a complex-state instance (entered
    on its own); the batch's second zero-guess solve runs the schedule
    predicted from the first."""
    import torch
    from paper_2603_04350_amd import Batch, Solver
    insts = W.batch(10, seed=4, ns=(16, 32, 64), nts=(8, 16, 32),
                    precision=1)
    for i, inst in enumerate(insts):
        inst.precision = i % 2
    solvers = [Solver.from_instance(i) for i in insts]
    cs, csh = _cstate_solver()
    solvers.append(cs)
    u0s = [_dev(i.u0) for i in insts] + [_dev(_cstate_u0())]
    shapes = [(_shape(i), torch.float64) for i in insts]
    shapes.append((csh, torch.complex128))
    b = Batch(solvers)
    Us = [_full(sh, 0.0, dt) for sh, dt in shapes]
    rc, its, rels, sts = b.iterate(u0s, Us, max_iter=200, tol=1e-12)
    ref = [U.cpu().numpy() for U in Us]
    b.set_zero_guess(True)
    nan = float("nan")
    for _ in range(2):
        Us = [_full(sh, complex(nan, nan) if dt == torch.complex128 else nan,
                    dt) for sh, dt in shapes]
        rc2, its2, rels2, sts2 = b.iterate(u0s, Us, max_iter=200, tol=1e-12)
        assert its2 == its and sts2 == sts
        for k, U in enumerate(Us):
            assert np.array_equal(U.cpu().numpy(), ref[k]), k
    b.close()
    for s in solvers:
        s.close()


def test_zero_guess_solve_stopped_before_the_fp64_phase():
    """A mixed instance that keeps its bulk iterate in fp32 is not given a
    cleared fp64 iterate by the zero-guess entry: the switch iteration writes
    all of it, or, when max_iter stops the solve in the bulk phase or at the
    switch, the exit widens the fp32 iterate into it.  Every cap from 1 to 12
    iterations (the fp64 phase starts within them), after a solve that left
    its converged fp64 iterate in the handle, against the same capped solve
    from a zeroed U."""
    from paper_2603_04350_amd import Solver
    inst, prec = SINGLE["ac2d_mixed_bulk_fp32"]
    u0 = _dev(inst.u0)
    with Solver.from_instance(inst, precision=prec) as s:
        for cap in range(1, 13):
            s.set_zero_guess(False)
            U = _full(_shape(inst), 0.0)
            rc, it, rel = s.iterate(u0, U, max_iter=cap, tol=1e-12)
            ref = U.cpu().numpy()
            s.iterate(u0, _full(_shape(inst), 0.0), max_iter=200, tol=1e-12)
            s.set_zero_guess(True)
            U = _full(_shape(inst), float("nan"))
            assert s.iterate(u0, U, max_iter=cap, tol=1e-12) == (rc, it, rel)
            assert np.array_equal(U.cpu().numpy(), ref), cap


def test_batch_zero_guess_stopped_before_the_fp64_phase():
    """The batch form of the test above: mixed instances capped at 1 to 8
    iterations each, after a batch solve that left converged fp64 iterates
    in every handle."""
    from paper_2603_04350_amd import Batch, Solver
    insts = W.batch(8, seed=5, ns=(16, 32), nts=(8, 16), precision=1)
    solvers = [Solver.from_instance(i) for i in insts]
    u0s = [_dev(i.u0) for i in insts]
    b = Batch(solvers)
    caps = [1 + k for k in range(len(insts))]
    tols = [0.0] * len(insts)
    Us = [_full(_shape(i), 0.0) for i in insts]
    out = b.iterate_each(u0s, Us, caps, tols)
    ref = [U.cpu().numpy() for U in Us]
    b.iterate(u0s, [_full(_shape(i), 0.0) for i in insts], max_iter=200,
              tol=1e-12)
    b.set_zero_guess(True)
    Us = [_full(_shape(i), float("nan")) for i in insts]
    assert b.iterate_each(u0s, Us, caps, tols) == out
    for k, U in enumerate(Us):
        assert np.array_equal(U.cpu().numpy(), ref[k]), k
    b.close()
    for s in solvers:
        s.close()
