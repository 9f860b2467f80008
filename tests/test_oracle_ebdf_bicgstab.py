"""Pins of the oracle's exponential BDF3..6 path (Sec. bdfs) and of its
BiCGStab (Table cpu_time_combined).

Independent references:
  * the BDF coefficients from the backward-difference definition of the
    order-s BDF formula (sum_{k=1..s} nabla^k / k), in exact fractions;
  * the exactness of the exponential BDF on u_n = A^n u_0 (the coefficients
    sum to one and the start values are exact);
  * the all-at-once systems assembled entry by entry (alpha entries where
    the paper lists them), solved by dense LU, with f_s written row by row
    as the paper prints it;
  * C_{j-1}^alpha = (C_0^alpha)^j as a matrix identity, and the rank of
    R^alpha - R (at most s eigenvalues per spatial mode of the preconditioned
    operator differ from one);
  * scipy's BiCGStab on the same operator (iterate by iterate), and dense
    solves.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle as O

ORDERS = [3, 4, 5, 6]
SCHEME = {3: O.EBDF3, 4: O.EBDF4, 5: O.EBDF5, 6: O.EBDF6}


def _setup(s, dim=1, n=8, Nt=12, dt=0.1, alpha=0.05, a=0.3, **kw):
    return O.Setup(dim, n, Nt, dt, alpha, a=a, scheme=SCHEME[s], **kw)


def _u0(st, seed=0):
    return np.random.default_rng([seed, st.n, st.Nt]).uniform(
        -0.9, 0.9, size=(st.n,) * st.dim)


def _bdf_from_differences(s):
    """beta_j of y_n = sum_j beta_j y_{n-j} + h b f_n from
    sum_{k=1..s} (1/k) nabla^k y_n = h f_n."""
    c = [Fraction(0)] * (s + 1)
    for k in range(1, s + 1):
        for i in range(k + 1):
            c[i] += Fraction((-1) ** i * math.comb(k, i), k)
    return [-c[j] / c[0] for j in range(1, s + 1)]


@pytest.mark.parametrize("s", [2] + ORDERS)
def test_coefficients_are_the_bdf_coefficients(s):
    num, den = O.EBDF_COEFFS[s]
    assert [Fraction(b, den) for b in num] == _bdf_from_differences(s)
    assert O.ebdf_beta(s) == [b / den for b in num]


@pytest.mark.parametrize("s", ORDERS)
def test_order_codes(s):
    assert O.ebdf_order(SCHEME[s]) == s
    assert O.ebdf_order(O.EBDF2) == 2
    assert O.ebdf_order(1) == 0 and O.ebdf_order(O.IF1) == 0


@pytest.mark.parametrize("s", ORDERS)
@pytest.mark.parametrize("dim", [1, 2])
def test_sequential_is_exact_on_linear_problem(s, dim):
    """Every slice equals A^n u_0 = ifft(E^n fft(u_0))."""
    st = _setup(s, dim=dim, n=8, Nt=14, c=0.2)
    u0 = _u0(st)
    U = O.sequential_ebdf(st, u0)
    u0h = np.fft.fftn(u0)
    for m in range(st.Nt):
        ex = np.fft.ifftn(st.E ** (m + 1) * u0h).real
        assert np.max(np.abs(U[m] - ex)) < 1e-13


@pytest.mark.parametrize("s", ORDERS)
def test_parasitic_modes_decay(s):
    """Perturbed start values: the recurrence in one Fourier mode is the BDF
    characteristic recurrence scaled by E, whose extra roots lie inside the
    unit disc (zero stability of BDF up to order six), so the perturbation
    decays relative to E^n."""
    beta = O.ebdf_beta(s)
    roots = np.roots([1.0] + [-b for b in beta])
    extra = sorted(np.abs(roots))[:-1]
    assert abs(sorted(np.abs(roots))[-1] - 1.0) < 1e-12
    assert max(extra) < 1.0


def _fs_rows(s, Ap, start):
    """f_s as printed for s = 3..6: row i is
    sum_{j=i+1..s} beta_j A^j u_{s+i-j}, rows s.. zero."""
    beta = O.ebdf_beta(s)
    rows = []
    for i in range(s):
        acc = 0.0
        for j in range(i + 1, s + 1):
            acc = acc + beta[j - 1] * (Ap[j] @ start[s + i - j])
        rows.append(acc)
    return rows


@pytest.mark.parametrize("s", ORDERS)
def test_f3_matches_printed_rows(s):
    """For s = 3 the rows of f_3 are the paper's three nonzero rows."""
    st = _setup(s, Nt=12)
    D = O.dense_operators_ebdf(st)
    u0 = _u0(st).ravel()
    start = [np.linalg.matrix_power(D["A"], j) @ u0 for j in range(s)]
    rows = _fs_rows(s, D["Ap"], start)
    if s == 3:
        A, A2, A3 = D["Ap"][1], D["Ap"][2], D["Ap"][3]
        u1, u2 = start[1], start[2]
        printed = [18 / 11 * A @ u2 - 9 / 11 * A2 @ u1 + 2 / 11 * A3 @ u0,
                   -9 / 11 * A2 @ u2 + 2 / 11 * A3 @ u1,
                   2 / 11 * A3 @ u2]
        for r, p in zip(rows, printed):
            assert np.max(np.abs(r - p)) < 1e-14
    zeros = np.zeros((st.Nt, st.n))
    R = O.residual_ebdf(st, u0.reshape(st.n), zeros)
    o = s - 1
    for i in range(s):
        assert np.max(np.abs(R[o + i] - rows[i])) < 1e-13
    assert np.max(np.abs(R[o + s:])) == 0.0


@pytest.mark.parametrize("s", ORDERS)
def test_alpha_circulants_are_powers(s):
    """The alpha entries the paper lists make C_{j-1}^alpha the j-th power of
    C_0^alpha, so all of them are diagonalised by Gamma_alpha and F with
    eigenvalues lambda_{0,m}^j."""
    st = _setup(s, Nt=16, alpha=0.3)
    D = O.dense_operators_ebdf(st)
    N = st.Nt - s + 1
    C0a = D["Ca"][0]
    for j in range(1, s + 1):
        assert np.array_equal(D["Ca"][j - 1],
                              np.linalg.matrix_power(C0a, j))
    gamma, lams = O.ebdf_tables(st, s)
    G = np.diag(gamma)
    l = np.arange(N)
    F = np.exp(2j * np.pi * np.outer(l, l) / N) / np.sqrt(N)
    for j in range(1, s + 1):
        M = F @ G @ D["Ca"][j - 1] @ np.linalg.inv(G) @ F.conj().T
        assert np.max(np.abs(M - np.diag(lams[j - 1]))) < 1e-12


@pytest.mark.parametrize("s", ORDERS)
def test_paper_positions_of_alpha(s):
    """Positions printed for C_2..C_5 (1-based, in terms of Nt, for the
    order whose system has N = Nt - s + 1 rows): C_{s-1}(i, Nt - 2(s-1) +
    i - 1) = alpha, i = 1..s."""
    st = _setup(s, Nt=20, alpha=0.25)
    D = O.dense_operators_ebdf(st)
    Ca = D["Ca"][s - 1]
    N = st.Nt - s + 1
    for i in range(1, s + 1):
        col = st.Nt - 2 * (s - 1) + i - 1
        assert Ca[i - 1, col - 1] == st.alpha
    assert np.count_nonzero(Ca == st.alpha) == s
    assert np.count_nonzero(Ca) == N


@pytest.mark.parametrize("s", ORDERS)
@pytest.mark.parametrize("dim", [1, 2])
def test_residual_and_operators_match_dense(s, dim):
    n = 8 if dim == 1 else 4
    st = _setup(s, dim=dim, n=n, Nt=11, c=0.1)
    D = O.dense_operators_ebdf(st)
    o = s - 1
    N = st.Nt - o
    rng = np.random.default_rng(3)
    V = rng.standard_normal((N,) + (n,) * dim)
    Rv = O.r_apply_ebdf(st, V)
    assert np.max(np.abs(Rv.reshape(-1) - D["R"] @ V.reshape(-1))) < 1e-13
    Rav = O.ralpha_apply_ebdf(st, V)
    assert np.max(np.abs(Rav.reshape(-1) - D["Ra"] @ V.reshape(-1))) < 1e-13
    u0 = _u0(st)
    U = rng.standard_normal((st.Nt,) + (n,) * dim)
    R = O.residual_ebdf(st, u0, U)
    f = O.residual_ebdf(st, u0, np.zeros_like(U))[o:]
    assert np.max(np.abs((R[o:] - f).reshape(-1)
                         + D["R"] @ U[o:].reshape(-1))) < 1e-13
    for j in range(1, s):
        ex = np.linalg.matrix_power(D["A"], j) @ u0.reshape(-1)
        assert np.max(np.abs(R[j - 1].reshape(-1)
                             - (ex - U[j - 1].reshape(-1)))) < 1e-13


@pytest.mark.parametrize("s", ORDERS)
@pytest.mark.parametrize("alpha", [0.5, 1e-3])
def test_precond_is_dense_solve(s, alpha):
    st = _setup(s, n=8, Nt=13, alpha=alpha)
    D = O.dense_operators_ebdf(st)
    o = s - 1
    Rv = np.random.default_rng(4).standard_normal((st.Nt, st.n))
    S = O.precond_apply_ebdf(st, Rv)
    assert np.array_equal(S[:o], Rv[:o])
    ex = np.linalg.solve(D["Ra"], Rv[o:].reshape(-1))
    scale = np.max(np.abs(ex))
    assert np.max(np.abs(S[o:].reshape(-1) - ex)) < 1e-12 * max(1, scale) / \
        min(1.0, alpha ** 0.5)


@pytest.mark.parametrize("s", ORDERS)
def test_dense_solve_equals_sequential(s):
    st = _setup(s, dim=2, n=4, Nt=10, c=0.05)
    D = O.dense_operators_ebdf(st)
    u0 = _u0(st)
    o = s - 1
    f = O.residual_ebdf(st, u0, np.zeros((st.Nt,) + u0.shape))[o:]
    v = np.linalg.solve(D["R"], f.reshape(-1))
    ref = O.sequential_ebdf(st, u0)
    assert np.max(np.abs(v - ref[o:].reshape(-1))) < 1e-13


@pytest.mark.parametrize("s", ORDERS)
def test_rank_of_alpha_correction(s):
    """R^alpha - R has rank <= s per spatial mode, so at most s Ns
    eigenvalues of (R^alpha)^{-1} R differ from one."""
    st = _setup(s, n=4, Nt=12, alpha=0.2)
    D = O.dense_operators_ebdf(st)
    ev = np.linalg.eigvals(np.linalg.solve(D["Ra"], D["R"]))
    assert np.count_nonzero(np.abs(ev - 1.0) > 1e-8) <= s * st.n
    # and they are small perturbations of 1 for small alpha
    st2 = _setup(s, n=4, Nt=12, alpha=1e-4)
    D2 = O.dense_operators_ebdf(st2)
    ev2 = np.linalg.eigvals(np.linalg.solve(D2["Ra"], D2["R"]))
    assert np.max(np.abs(ev2 - 1.0)) < 1e-2


@pytest.mark.parametrize("s", ORDERS)
@pytest.mark.parametrize("dim", [1, 2])
def test_fixed_point_reaches_sequential(s, dim):
    n = 32 if dim == 1 else 8
    st = _setup(s, dim=dim, n=n, Nt=16, dt=0.05, alpha=1e-3, a=0.1)
    u0 = _u0(st)
    ref = O.sequential(st, u0)
    U, it, _ = O.fixed_point(st, u0, tol=1e-14, max_iter=100)
    assert O.rel_err(U, ref) < 1e-13, it
    assert it <= 6      # the error falls by about alpha per iteration


@pytest.mark.parametrize("s", ORDERS)
def test_fixed_point_error_contracts_like_alpha(s):
    """Smaller alpha, faster convergence (the behaviour Sec. bdfs and
    Theorem thm_bdf2 describe): iterations to 1e-12 fall with alpha."""
    its = []
    for alpha in (1e-1, 1e-2, 1e-4):
        st = _setup(s, n=16, Nt=20, dt=0.05, alpha=alpha, a=0.1)
        u0 = _u0(st)
        ref = O.sequential(st, u0)
        _, it, _ = O.fixed_point(st, u0, ref=ref, ref_tol=1e-12,
                                 max_iter=200)
        its.append(it)
    assert its[0] > its[1] > its[2], its


@pytest.mark.parametrize("s", ORDERS)
def test_gmres_reaches_sequential(s):
    st = _setup(s, n=32, Nt=20, dt=0.05, alpha=1e-2, a=1e-5)
    u0 = _u0(st)
    U, it, hist = O.gmres_solve_ebdf(st, u0, restart=20, tol=1e-13)
    assert O.rel_err(U, O.sequential(st, u0)) < 1e-12
    assert it <= 10


def test_generic_order_two_is_ebdf2():
    st = O.Setup(1, 16, 9, 0.1, 0.05, a=0.2, scheme=O.EBDF2)
    u0 = _u0(st)
    rng = np.random.default_rng(6)
    U = rng.standard_normal((st.Nt, st.n))
    assert np.max(np.abs(O.sequential_ebdf(st, u0, 2)
                         - O.sequential_ebdf2(st, u0))) < 1e-14
    assert np.max(np.abs(O.residual_ebdf(st, u0, U, 2)
                         - O.residual_ebdf2(st, u0, U))) < 1e-13
    assert np.max(np.abs(O.precond_apply_ebdf(st, U, 2)
                         - O.precond_apply_ebdf2(st, U))) < 1e-12


# --------------------------------------------------------------- BiCGStab
def test_bicgstab_dense_system():
    rng = np.random.default_rng(7)
    n = 40
    M = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, it, hist = O.bicgstab(lambda v: M @ v, b, np.zeros(n), tol=1e-14,
                             max_iter=200)
    assert np.max(np.abs(x - np.linalg.solve(M, b))) < 1e-12
    assert hist[-1] <= 1e-14 * np.linalg.norm(b)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_bicgstab_iterates_match_scipy(k):
    from scipy.sparse.linalg import bicgstab as sp_bicgstab
    rng = np.random.default_rng(8)
    n = 30
    M = np.eye(n) + 0.5 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x0 = 0.1 * rng.standard_normal(n)
    x, it, _ = O.bicgstab(lambda v: M @ v, b, x0, tol=0.0, max_iter=k)
    xs, info = sp_bicgstab(M, b, x0=x0, rtol=0.0, atol=0.0, maxiter=k)
    assert it == k
    assert np.max(np.abs(x - xs)) < 1e-12 * max(1.0, np.max(np.abs(xs)))


def test_bicgstab_one_step_for_scaled_identity():
    b = np.arange(1.0, 6.0)
    x, it, _ = O.bicgstab(lambda v: 2.5 * v, b, np.zeros(5), tol=1e-15)
    assert it == 1 and np.max(np.abs(x - b / 2.5)) < 1e-15


@pytest.mark.parametrize("scheme,dim,n,Nt", [(1, 1, 32, 16), (1, 2, 8, 8),
                                             (O.EBDF2, 1, 32, 17),
                                             (O.EBDF4, 1, 32, 19)])
def test_bicgstab_solve_reaches_sequential(scheme, dim, n, Nt):
    st = O.Setup(dim, n, Nt, 0.05, 1e-2, a=0.1, scheme=scheme)
    u0 = np.random.default_rng(9).uniform(-1, 1, (n,) * dim)
    U, it, hist = O.bicgstab_solve(st, u0, tol=1e-13)
    assert O.rel_err(U, O.sequential(st, u0)) < 1e-12
    assert it <= 10


def test_bicgstab_complex_state():
    st = O.Setup(1, 32, 16, 1.0 / 16, 1e-2, a=0.0, a_im=1.0, c_im=2.0)
    rng = np.random.default_rng(10)
    u0 = rng.uniform(-1, 1, 32) + 1j * rng.uniform(-1, 1, 32)
    U, it, _ = O.bicgstab_solve(st, u0, tol=1e-13)
    assert O.rel_err(U, O.sequential(st, u0)) < 1e-12


@pytest.mark.parametrize("scheme", [1, 2])
def test_newton_bicgstab_reaches_dense_newton(scheme):
    st = O.Setup(1, 16, 8, 0.05, 1e-2, a=0.01, n1=1.0, n3=-1.0,
                 scheme=scheme)
    u0 = np.random.default_rng(11).uniform(-0.9, 0.9, 16)
    U, newton, inner, hist = O.newton_bicgstab(st, u0, tol=1e-12)
    assert O.rel_err(U, O.dense_newton(st, u0)) < 1e-11
    assert O.rel_err(U, O.sequential(st, u0)) < 1e-11


# --------------------------------------------------- printed values (golden)
import os  # noqa: E402
import re  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.strip() for l in f if l.strip() and not l.startswith("#")]


def test_printed_coefficients_match_bdf_and_oracle():
    """The paper's printed beta_i (tests/golden/ebdf_coefficients.txt) are
    the BDF coefficients of the backward-difference definition, and the
    oracle uses them."""
    for line in _golden_lines("ebdf_coefficients.txt"):
        s, rest = line.split(":")
        s = int(s)
        printed = [Fraction(t) for t in rest.split()]
        assert printed == _bdf_from_differences(s), s
        num, den = O.EBDF_COEFFS[s]
        assert printed == [Fraction(b, den) for b in num], s


@pytest.mark.parametrize("Nt", [14, 20, 31])
def test_printed_alpha_positions_match_oracle(Nt):
    """Each alpha-circulant C_j^alpha the paper lists, in the system of the
    order whose dimension N = Nt - s + 1 it fits, has alpha exactly at the
    printed (row, Nt - k) entries, as the oracle assembles it."""
    for line in _golden_lines("alpha_circulant_positions.txt"):
        head, rest = line.split(":")
        name, s = head.split()
        j, s = int(name[1:]), int(s)
        pos = [(int(r), Nt - int(k)) for r, k in
               re.findall(r"\((\d+), Nt-(\d+)\)", rest)]
        assert len(pos) == j + 1
        st = _setup(s, Nt=Nt, alpha=0.25)
        Ca = O.dense_operators_ebdf(st)["Ca"][j]
        got = [(int(r) + 1, int(c) + 1)
               for r, c in zip(*np.nonzero(Ca == st.alpha))]
        assert sorted(got) == sorted(pos), (name, s, got, pos)
