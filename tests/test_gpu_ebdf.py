"""GPU exponential BDF3..6 windows (Sec. bdfs) vs the CPU oracle, element by
element, through the C ABI.

Tolerances as for EBDF2: the residual is a few FFT roundings (1e-13
relative); the preconditioner and the iterates carry the conditioning of the
alpha-scaled time diagonalisation, roughly eps/alpha, and, on the oracle's
side, the rounding of its step (b) symbol d = 1 - sum_j beta_j lambda^j E^j
evaluated as written: absolute error about eps sum_j |beta_j|, relative
eps sum_j |beta_j| / |d| (sum |beta_j| is 10.3 for order six, and |d| is
smallest, about (1 - alpha^{1/N}) q(1), for the lowest modes).  The kernel
evaluates d factored as (1 - z) q(z).  Their bar is max(1e-12,
50 eps / alpha, 10 eps sum_j |beta_j| / min |d|) relative; converged
windows are held to 1e-12 against sequential stepping of the same scheme.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

EPS = 2.220446049250313e-16
SCHEME = {3: O.EBDF3, 4: O.EBDF4, 5: O.EBDF5, 6: O.EBDF6}

# (s, dim, n, Nt, alpha, a, c, b): ragged kappa tiles; both time transforms
# (dense: Nt a power of two 8..128; radix FFT: Nt - s + 1 a power of two
# 2..512) at their smallest and largest sizes
CASES = {
    "s3_dense_heat1d_Nt16": (3, 1, 64, 16, 1e-2, 1.0, 0.0, None),
    "s4_dense_heat2d_Nt32": (4, 2, 16, 32, 1e-3, 0.3, 0.2, None),
    "s5_dense_heat3d_Nt8_min": (5, 3, 8, 8, 0.2, 0.5, 0.1, None),
    "s6_dense_heat1d_Nt8": (6, 1, 32, 8, 1e-2, 0.3, 0.0, None),
    "s6_dense_heat2d_Nt128_max": (6, 2, 8, 128, 1e-2, 0.05, 0.0, None),
    "s3_fft_heat1d_Nt18": (3, 1, 64, 18, 1e-2, 1.0, 0.0, None),
    "s4_fft_heat2d_Nt67": (4, 2, 16, 67, 1e-3, 0.3, 0.2, None),
    "s5_fft_heat1d_Nt6_min": (5, 1, 16, 6, 0.2, 0.5, 0.1, None),
    "s6_fft_heat3d_Nt13": (6, 3, 8, 13, 1e-3, 1.0, 0.0, None),
    "s6_fft_heat2d_Nt517_max": (6, 2, 8, 517, 1e-2, 0.01, 0.0, None),
    "s3_fft_advection2d_Nt18": (3, 2, 16, 18, 1e-3, 0.05, 0.0, (2.0, 1.0)),
    "s5_dense_advection1d_Nt32": (5, 1, 64, 32, 1e-2, 0.1, 0.0, (2.0,)),
}


def _setup(case, T=1.0):
    s, dim, n, Nt, alpha, a, c, b = CASES[case]
    bb = tuple(b or ()) + (0.0,) * (3 - len(b or ()))
    return O.Setup(dim, n, Nt, T / Nt, alpha, a, c, scheme=SCHEME[s], b=bb)


def _u0(st, seed=0):
    rng = np.random.default_rng([seed, st.n, st.Nt, 5])
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
                  st.a, st.c, 0.0, 0.0, 0.0, 0, restart, b=st.b)


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _bar(st):
    s = O.ebdf_order(st.scheme)
    beta = O.ebdf_beta(s)
    lam0 = O.ebdf_tables(st, s)[1][0]
    z = lam0.reshape(-1, 1) * st.E.reshape(1, -1)
    d = 1.0 - sum(beta[j - 1] * z ** j for j in range(1, s + 1))
    floor = 10 * EPS * sum(abs(b) for b in beta) / np.abs(d).min()
    return max(1e-12, 50 * EPS / st.alpha, floor)


@pytest.mark.parametrize("case", sorted(CASES))
def test_ebdf_residual_parity(case):
    import torch
    st = _setup(case)
    u0 = _u0(st)
    U = 0.5 * np.random.default_rng(1).standard_normal(
        (st.Nt,) + (st.n,) * st.dim)
    with _solver(st) as s:
        R = torch.empty_like(_dev(U))
        rn = s.residual(_dev(u0), _dev(U), R)
        torch.cuda.synchronize()
    Rr = O.residual_ebdf(st, u0, U)
    assert _rel(R.cpu().numpy(), Rr) < 1e-13
    assert abs(rn - np.linalg.norm(Rr)) < 1e-12 * np.linalg.norm(Rr)


@pytest.mark.parametrize("case", sorted(CASES))
def test_ebdf_precond_parity(case):
    import torch
    st = _setup(case)
    Rv = np.random.default_rng(2).standard_normal((st.Nt,) + (st.n,) * st.dim)
    with _solver(st) as s:
        S = torch.empty_like(_dev(Rv))
        s.precond_apply(_dev(Rv), S)
        torch.cuda.synchronize()
        Sg = S.cpu().numpy()
        # in place: R and S the same buffer
        T = _dev(Rv)
        s.precond_apply(T, T)
        torch.cuda.synchronize()
    Sr = O.precond_apply_ebdf(st, Rv)
    assert _rel(Sg, Sr) < _bar(st)
    assert np.array_equal(T.cpu().numpy(), Sg)


@pytest.mark.parametrize("case", sorted(CASES))
def test_ebdf_iterates_parity(case):
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


def test_ebdf_iterates_ignore_initial_start_slices():
    """f_s takes the start values A^m u0, not what the start slices of the
    initial iterate hold; after one iteration they hold A^m u0."""
    st = _setup("s5_fft_heat1d_Nt6_min")
    u0 = _u0(st)
    U0 = np.zeros((st.Nt,) + (st.n,) * st.dim)
    U0[:4] = np.random.default_rng(9).standard_normal((4, st.n))
    ref, _, _ = O.fixed_point(st, u0, max_iter=1, tol=0.0)  # from zeros
    with _solver(st) as s:
        U = _dev(U0)
        s.iterate(_dev(u0), U, max_iter=1, tol=0.0)
    assert O.rel_err(U.cpu().numpy(), ref) < _bar(st)


@pytest.mark.parametrize("case", sorted(CASES))
def test_ebdf_converged_equals_sequential(case):
    st = _setup(case)
    u0 = _u0(st)
    ref = O.sequential(st, u0)
    with _solver(st) as s:
        U = _zeros(st)
        rc, it, rel = s.iterate(_dev(u0), U, max_iter=300, tol=1e-14)
    err = O.rel_err(U.cpu().numpy(), ref)
    assert err < 1e-12, (it, rel, err)


@pytest.mark.parametrize("case", ["s3_dense_heat1d_Nt16", "s4_fft_heat2d_Nt67",
                                  "s6_fft_heat3d_Nt13",
                                  "s3_fft_advection2d_Nt18"])
def test_ebdf_gmres_solution(case):
    st = _setup(case)
    u0 = _u0(st)
    ref = O.sequential(st, u0)
    with _solver(st, restart=20) as s:
        U = _zeros(st)
        rc, it, rel = s.gmres(_dev(u0), U, restart=20, max_iter=200,
                              tol=1e-13)
    assert rel <= 1e-13
    assert O.rel_err(U.cpu().numpy(), ref) < 1e-12
    # the oracle's GMRES on the same system takes as many iterations
    _, it_o, _ = O.gmres_solve_ebdf(st, u0, restart=20, tol=1e-13)
    assert abs(it - it_o) <= 1, (it, it_o)


@pytest.mark.parametrize("case,variant", [("s4_dense_heat2d_Nt32", 1),
                                          ("s4_fft_heat2d_Nt67", 0)])
def test_ebdf_variant_and_autotune(case, variant):
    from paper_2603_04350_amd import expdiag as X
    st = _setup(case)
    with _solver(st) as s:
        assert X.expdiag_get_time_variant(s.h) == variant
        with pytest.raises(RuntimeError):
            X.expdiag_set_time_variant(s.h, 1 - variant)
        v, tf, td = X.expdiag_autotune(s.h, None)
        assert v == variant
        assert (tf > 0 and td == -1) if variant == 0 else \
            (tf == -1 and td > 0)


def test_ebdf_orders_in_one_batch():
    """EBDF3, EBDF5 and EBDF6 windows (radix kernels of their own order,
    and the dense kernel that reads the order per job) with EBDF2 and ETD1
    instances in one batch: every result is bitwise the one its handle
    gives alone."""
    import torch
    from paper_2603_04350_amd import Batch, Solver
    sts = [O.Setup(2, 16, 18, 1.0 / 18, 1e-3, 0.3, 0.1, scheme=O.EBDF3),
           O.Setup(2, 16, 20, 1.0 / 20, 1e-3, 0.3, 0.1, scheme=O.EBDF5),
           O.Setup(1, 64, 32, 1.0 / 32, 1e-2, 0.2, scheme=O.EBDF6),
           O.Setup(1, 64, 17, 1.0 / 17, 1e-2, 0.2, scheme=O.EBDF2)]
    solvers = [_solver(st) for st in sts]
    u0s = [_u0(st, 3) for st in sts]
    etd = O.Setup(2, 32, 16, 1.0 / 16, 1e-3, a=0.0025, n1=1.0, n3=-1.0)
    solvers.append(Solver((32, 32), 16, etd.dt, etd.alpha, 1, etd.a, 0.0,
                          1.0, 0.0, -1.0))
    u0s.append(np.random.default_rng(7).uniform(-0.9, 0.9, (32, 32)))
    shapes = [(st.Nt,) + (st.n,) * st.dim for st in sts] + [(16, 32, 32)]
    solo = []
    for s, u0, sh in zip(solvers, u0s, shapes):
        U = torch.zeros(sh, dtype=torch.float64, device="cuda:0")
        s.iterate(_dev(u0), U, max_iter=200, tol=1e-12)
        solo.append(U.cpu().numpy())
    b = Batch(solvers)
    Us = [torch.zeros(sh, dtype=torch.float64, device="cuda:0")
          for sh in shapes]
    b.iterate([_dev(u) for u in u0s], Us, max_iter=200, tol=1e-12)
    b.close()
    for k in range(len(Us)):
        assert np.array_equal(Us[k].cpu().numpy(), solo[k]), k
    for k, st in enumerate(sts):
        assert O.rel_err(solo[k], O.sequential(st, u0s[k])) < 1e-11
    for s in solvers:
        s.close()


def test_ebdf_complex_state():
    """A Schroedinger window (a = i, complex state, full spectrum) stepped by
    EBDF4."""
    st = O.Setup(1, 32, 19, 1.0 / 19, 1e-3, a=0.0, a_im=1.0, c_im=2.0,
                 scheme=O.EBDF4)
    rng = np.random.default_rng(12)
    u0 = rng.uniform(-0.9, 0.9, 32) + 1j * rng.uniform(-0.9, 0.9, 32)
    import torch
    from paper_2603_04350_amd import Solver
    with Solver((32,), st.Nt, st.dt, st.alpha, st.scheme, 0.0, 0.0,
                a_im=1.0, c_im=2.0, complex_state=1) as s:
        R = torch.empty((st.Nt, 32), dtype=torch.complex128, device="cuda:0")
        Ur = rng.standard_normal((st.Nt, 32)) + 1j * rng.standard_normal(
            (st.Nt, 32))
        s.residual(torch.from_numpy(u0).to("cuda:0"),
                   torch.from_numpy(Ur).to("cuda:0"), R)
        torch.cuda.synchronize()
        assert _rel(R.cpu().numpy(), O.residual_ebdf(st, u0, Ur)) < 1e-13
        U = torch.zeros((st.Nt, 32), dtype=torch.complex128, device="cuda:0")
        s.iterate(torch.from_numpy(u0).to("cuda:0"), U, max_iter=100,
                  tol=1e-14)
    assert O.rel_err(U.cpu().numpy(), O.sequential(st, u0)) < 1e-12


def test_server_reuses_or_rebuilds_pooled_handles():
    """The server pools finished handles by grid and Nt and re-initialises
    them for the next request.  An EBDF6 handle with Nt = 9 (4 transform
    points) is too small for EBDF2 at Nt = 9 (8 points) and is rebuilt; the
    EBDF2 handle then serves EBDF6.  Every result equals the solo one."""
    import time
    import torch
    from paper_2603_04350_amd import expdiag as X
    sts = [O.Setup(1, 64, 9, 0.1, 1e-2, 0.3, scheme=O.EBDF6),
           O.Setup(1, 64, 9, 0.1, 1e-2, 0.3, scheme=O.EBDF2),
           O.Setup(1, 64, 9, 0.1, 1e-2, 0.3, scheme=O.EBDF6)]
    srv = X.expdiag_server_create(1 << 30, 1)
    try:
        for k, st in enumerate(sts):
            u0 = _u0(st, k)
            solo = _zeros(st)
            with _solver(st) as s:
                s.iterate(_dev(u0), solo, max_iter=100, tol=1e-13)
            U = _zeros(st)
            du0 = _dev(u0)
            torch.cuda.synchronize()
            rid = X.expdiag_server_submit(srv, (64,), 9, 0.1, 1e-2, st.scheme,
                                          X.make_problem(0.3), du0, U, 100,
                                          1e-13)
            done = []
            t_end = time.time() + 30
            while not done and time.time() < t_end:
                res, _ = X.expdiag_server_poll(srv)
                done.extend(r for r in res if r["id"] == rid)
                time.sleep(0.001)
            assert done and done[0]["status"] == 0, done
            assert np.array_equal(U.cpu().numpy(), solo.cpu().numpy()), k
            assert O.rel_err(U.cpu().numpy(), O.sequential(st, u0)) < 1e-12
    finally:
        X.expdiag_server_destroy(srv)
