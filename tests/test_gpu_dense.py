"""Dense-MFMA time transform and the autotuner, through the C ABI.

The dense variant applies the same operator as the radix-FFT variant with
another rounding order, so it meets the same bars against the oracle
(max(1e-12, 50 eps/alpha) per apply, 1e-12 at convergence in fp64).
"""
import json

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

EPS = 2.220446049250313e-16

CASES = {
    "heat1d_Nt16": (1, 64, 16, 1e-2, 1.0, 0.0, 0, 0, 0, 1),
    "ac2d_Nt8_ragged": (2, 8, 8, 1e-3, 0.0025, 0.0, 1.0, 0, -1.0, 1),
    "ac2d_Nt32": (2, 32, 32, 1e-3, 0.0025, 0.0, 1.0, 0, -1.0, 1),
    "ac2d_Nt16_tiles": (2, 64, 16, 1e-2, 0.0025, 0.0, 1.0, 0, -1.0, 1),
    "rd2d_etd2_Nt64": (2, 32, 64, 1e-3, 0.1, 0.0, 1.0, 0, -1.0, 2),
    "heat3d_Nt128": (3, 8, 128, 1e-2, 1.0, 0.1, 0, 0, 0, 1),
}


def _setup(case, T=1.0):
    dim, n, Nt, alpha, a, c, n1, n2, n3, scheme = CASES[case]
    return O.Setup(dim, n, Nt, T / Nt, alpha, a, c, n1, n2, n3, scheme)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(
        "cuda:0")


def _solver(st, precision=0):
    from paper_2603_04350_amd import Solver
    from paper_2603_04350_amd import expdiag as X
    s = Solver((st.n,) * st.dim, st.Nt, st.dt, st.alpha, st.scheme, st.a,
               st.c, st.n1, st.n2, st.n3, precision)
    X.expdiag_set_time_variant(s.h, X.TIME_DENSE_MFMA)
    assert X.expdiag_get_time_variant(s.h) == X.TIME_DENSE_MFMA
    return s


@pytest.mark.parametrize("case", sorted(CASES))
def test_dense_precond_parity(case):
    import torch
    st = _setup(case)
    Rv = np.random.default_rng(2).standard_normal((st.Nt,) + (st.n,) * st.dim)
    with _solver(st) as s:
        S = torch.empty_like(_dev(Rv))
        s.precond_apply(_dev(Rv), S)
        torch.cuda.synchronize()
    Sr = O.precond_apply(st, Rv)
    err = np.max(np.abs(S.cpu().numpy() - Sr)) / np.max(np.abs(Sr))
    assert err < max(1e-12, 50 * EPS / st.alpha), err


@pytest.mark.parametrize("case", sorted(CASES))
def test_dense_iterate_converges_to_sequential(case):
    import torch
    st = _setup(case)
    u0 = np.random.default_rng([st.n, st.Nt]).uniform(-0.9, 0.9,
                                                      (st.n,) * st.dim)
    ref = O.sequential(st, u0)
    _, _, (_, its) = O.fixed_point(st, u0, max_iter=2, tol=0.0, record=True)
    with _solver(st) as s:
        U = torch.zeros((st.Nt,) + (st.n,) * st.dim, dtype=torch.float64,
                        device="cuda:0")
        s.iterate(_dev(u0), U, max_iter=2, tol=0.0)
        assert O.rel_err(U.cpu().numpy(), its[1]) < max(1e-12, 50 * EPS /
                                                       st.alpha)
        U.zero_()
        rc, it, rel = s.iterate(_dev(u0), U, max_iter=400, tol=1e-14)
    assert O.rel_err(U.cpu().numpy(), ref) < 1e-12


def test_dense_in_batch_with_fft_instances():
    """A batch mixing both variants: each instance equals its solo solve."""
    import torch
    from paper_2603_04350_amd import Batch, Solver
    from paper_2603_04350_amd import expdiag as X
    insts = W.batch(6, seed=2, ns=(16, 32), nts=(16, 32), precision=1)
    solvers = [Solver.from_instance(i) for i in insts]
    for k, s in enumerate(solvers):
        X.expdiag_set_time_variant(s.h, k % 2)
    solo = []
    for s, inst in zip(solvers, insts):
        U = torch.zeros((inst.Nt,) + inst.shape, dtype=torch.float64,
                        device="cuda:0")
        s.iterate(_dev(inst.u0), U, max_iter=300, tol=1e-12)
        solo.append(U.cpu().numpy())
    b = Batch(solvers)
    Us = [torch.zeros((i.Nt,) + i.shape, dtype=torch.float64,
                      device="cuda:0") for i in insts]
    b.iterate([_dev(i.u0) for i in insts], Us, max_iter=300, tol=1e-12)
    b.close()
    for k in range(len(insts)):
        assert np.array_equal(Us[k].cpu().numpy(), solo[k])
    for s in solvers:
        s.close()


def test_autotune_writes_and_reuses_cache(tmp_path):
    from paper_2603_04350_amd import Solver
    from paper_2603_04350_amd import expdiag as X
    inst = W.scaled(W.allen_cahn2d(), n=64, Nt=32)
    cache = tmp_path / "tune.json"
    with Solver.from_instance(inst) as s:
        v, tf, td = X.expdiag_autotune(s.h, cache)
        assert v in (0, 1) and tf > 0 and td > 0
        assert X.expdiag_get_time_variant(s.h) == v
    data = json.loads(cache.read_text())
    key = "gfx950/d2/64x64x1/Nt32/fp64"
    assert data[key]["variant"] == v
    with Solver.from_instance(inst) as s:
        v2, tf2, td2 = X.expdiag_autotune(s.h, cache)
        assert (v2, tf2, td2) == (v, data[key]["us_fft"],
                                  data[key]["us_dense"])


@pytest.mark.parametrize("case", ["ac2d_Nt32", "rd2d_etd2_Nt64",
                                  "heat3d_Nt128"])
def test_wide_columns_equal_default(case):
    """The 2C-column workgroups run the same column transforms: a mixed and
    an fp64 solve give the default's iterate bit for bit."""
    import torch
    from paper_2603_04350_amd import expdiag as X
    from paper_2603_04350_amd import Solver
    st = _setup(case)
    u0 = np.random.default_rng([st.n, st.Nt, 5]).uniform(-0.9, 0.9,
                                                         (st.n,) * st.dim)
    for prec in (0, 1):
        out = []
        for wide in (0, 1):
            with Solver((st.n,) * st.dim, st.Nt, st.dt, st.alpha, st.scheme,
                        st.a, st.c, st.n1, st.n2, st.n3, prec) as s:
                X.expdiag_set_tuning(s.h, 0, wide)
                assert X.expdiag_get_tuning(s.h) == (0, wide)
                U = torch.zeros((st.Nt,) + (st.n,) * st.dim,
                                dtype=torch.float64, device="cuda:0")
                rc, it, rel = s.iterate(_dev(u0), U, max_iter=300, tol=1e-12)
                out.append((it, U.cpu().numpy()))
        assert out[0][0] == out[1][0]
        assert np.array_equal(out[0][1], out[1][1])


def test_batch_autotune_then_solve(tmp_path):
    """A tuned batch (per-shape choices, graph replay or launches as
    measured) solves every instance to its solo result under the same
    tuning, and to the oracle's sequential stepping at the mixed bar."""
    import torch
    from paper_2603_04350_amd import Batch, Solver
    from paper_2603_04350_amd import expdiag as X
    insts = W.batch(8, seed=4, ns=(32, 64), nts=(16, 32), precision=1)
    solvers = [Solver.from_instance(i) for i in insts]
    b = Batch(solvers)
    u0s = [_dev(i.u0) for i in insts]
    Us = [torch.zeros((i.Nt,) + i.shape, dtype=torch.float64,
                      device="cuda:0") for i in insts]
    info = b.autotune(u0s, Us, tmp_path / "tune.json")
    shapes = {(i.n, i.Nt) for i in insts}
    assert info["shapes"] == len(shapes)
    assert info["ms_launch"] > 0
    assert info["graph_used"] == X.expdiag_batch_graph(b.b)
    for U in Us:
        assert float(U.abs().max()) == 0.0  # autotune reads U only
    data = json.loads((tmp_path / "tune.json").read_text())
    assert len(data) == len(shapes)
    rc, its, rels, sts = b.iterate(u0s, Us, max_iter=300, tol=1e-12)
    b.close()
    assert all(s == 0 for s in sts)
    for k, inst in enumerate(insts):
        V = torch.zeros_like(Us[k])
        solvers[k].iterate(u0s[k], V, max_iter=300, tol=1e-12)
        assert np.array_equal(V.cpu().numpy(), Us[k].cpu().numpy()), k
        ref = O.sequential(O.Setup.from_instance(inst), inst.u0)
        assert O.rel_err(Us[k].cpu().numpy(), ref) < 1e-10
    for s in solvers:
        s.close()


@pytest.mark.parametrize("case", ["ac2d_Nt32", "rd2d_etd2_Nt64"])
def test_dense_variant_residual_norm_and_newton_gmres(case):
    """A handle on the dense time transform runs the residual and the
    Krylov drivers' residual passes on the radix kernel: the residual and
    its norm match the oracle, and Newton-GMRES and Newton-BiCGStab reach
    sequential stepping."""
    import torch
    from paper_2603_04350_amd import Solver
    from paper_2603_04350_amd import expdiag as X
    st = _setup(case)
    rng = np.random.default_rng([st.n, st.Nt, 9])
    u0 = rng.uniform(-0.9, 0.9, (st.n,) * st.dim)
    Uv = 0.5 * rng.standard_normal((st.Nt,) + (st.n,) * st.dim)
    ref = O.sequential(st, u0)
    with Solver((st.n,) * st.dim, st.Nt, st.dt, st.alpha, st.scheme, st.a,
                st.c, st.n1, st.n2, st.n3, 0, 20) as s:
        X.expdiag_set_time_variant(s.h, X.TIME_DENSE_MFMA)
        R = torch.empty_like(_dev(Uv))
        rn = s.residual(_dev(u0), _dev(Uv), R)
        Rr = O.residual(st, u0, Uv)
        assert np.max(np.abs(R.cpu().numpy() - Rr)) / np.max(np.abs(Rr)) \
            < 1e-13
        assert abs(rn - np.linalg.norm(Rr)) < 1e-12 * np.linalg.norm(Rr)
        for solve in (s.gmres, s.bicgstab):
            U = torch.zeros((st.Nt,) + (st.n,) * st.dim, dtype=torch.float64,
                            device="cuda:0")
            rc, it, rel = solve(_dev(u0), U, max_iter=400, tol=1e-12)
            assert rel <= 1e-12
            assert O.rel_err(U.cpu().numpy(), ref) < 1e-10
