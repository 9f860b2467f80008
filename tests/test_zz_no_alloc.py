"""The no-allocation solve against the allocating one, through the C ABI.

expdiag_iterate_noalloc runs the fixed point of expdiag_iterate with every
device buffer carved from the library's fixed workspace; on the same inputs
it must give the same iterate (same kernels, same per-instance reduction
order), to the fp64 bar 1e-12, and it must stay correct when the workspace
holds a previous, larger call's contents.
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


def _zeros(inst):
    import torch
    return torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64,
                       device="cuda:0")


def _noalloc(inst, U, max_iter=300, tol=1e-12):
    from paper_2603_04350_amd import expdiag as X
    prob = X.make_problem(inst.a, inst.c, inst.n1, inst.n2, inst.n3,
                          inst.precision)
    return X.expdiag_iterate_noalloc(inst.shape, inst.Nt, inst.dt,
                                     inst.alpha, inst.scheme, prob,
                                     _dev(inst.u0), U, max_iter, tol)


def test_noalloc_equals_allocating_solve_twice():
    """Two calls in a row, the second smaller: the 256^2 x 64 Allen-Cahn
    headline instance in mixed precision (the workspace's largest 2D case),
    then a 64^2 x 16 ETD2 window in fp64; each equals the handle-based
    solve to 1e-12 and sequential stepping to the mixed / fp64 bar."""
    from paper_2603_04350_amd import Solver
    first = W.allen_cahn2d(precision=1)
    second = W.scaled(W.allen_cahn2d(precision=0), n=64, Nt=16)
    second.scheme = 2
    for inst, bar in ((first, 1e-10), (second, 1e-12)):
        U = _zeros(inst)
        rc, it, rel = _noalloc(inst, U)
        assert rc == 0, (inst.name, rc, it, rel)
        with Solver.from_instance(inst) as s:
            V = _zeros(inst)
            rc1, it1, rel1 = s.iterate(_dev(inst.u0), V, max_iter=300,
                                       tol=1e-12)
        # same iterations; the last update norm may differ in its last bit
        # (which kernel reduces the final iteration depends on where a
        # chunk ends)
        assert it == it1 and abs(rel - rel1) <= 1e-12 * rel1
        got = U.cpu().numpy()
        want = V.cpu().numpy()
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
        ref = O.sequential(O.Setup.from_instance(inst), inst.u0)
        assert O.rel_err(got, ref) < bar, (inst.name, O.rel_err(got, ref))


def test_noalloc_refuses_a_problem_beyond_its_workspace():
    """512^2 x 128 needs about 800 MB of handle buffers: refused with
    EINVAL, naming the sizes, before the device is touched."""
    from paper_2603_04350_amd import expdiag as X
    inst = W.rd2d()
    U = _zeros(inst)
    with pytest.raises(X.ExpdiagError) as ei:
        _noalloc(inst, U)
    assert ei.value.code == X.EXPDIAG_EINVAL
    assert "workspace" in str(ei.value)
    assert float(U.abs().max()) == 0.0
