"""Planted mistakes in the oracle must be caught by the pins.

Each test patches one plausible error into the CPU oracle (a swapped sign
pairing, a dropped Gamma_alpha, a conjugated eigenvalue, a dropped phi term,
an off-by-one in the time shift, a wrong symbol sign) and checks that at
least one pin of tests/test_oracle_pins.py then fails.  This is how we know
the pins constrain every part of the oracle.
"""
import numpy as np
import pytest

import oracle.expdiag_oracle as OE
import tests.test_oracle_pins as P


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    except (FloatingPointError, np.linalg.LinAlgError, ValueError,
            ZeroDivisionError, OverflowError):
        return True
    return False


def _patch_setup(monkeypatch, post):
    orig = OE.Setup.__post_init__

    def patched(self):
        orig(self)
        post(self)
    monkeypatch.setattr(OE.Setup, "__post_init__", patched)


def test_swapped_time_transform_sign(monkeypatch):
    dft, idft = OE.time_dft, OE.time_idft
    monkeypatch.setattr(OE, "time_dft", idft)
    monkeypatch.setattr(OE, "time_idft", dft)
    assert _fails(P.test_precond_apply_equals_dense_inverse, 1, 12, 8, 1e-2)


def test_dropped_gamma(monkeypatch):
    _patch_setup(monkeypatch, lambda s: setattr(s, "gamma",
                                                np.ones_like(s.gamma)))
    assert _fails(P.test_precond_apply_equals_dense_inverse, 1, 12, 8, 1e-2)
    assert _fails(P.test_alpha_circulant_diagonalisation, 8, 1e-2)


def test_conjugated_lambda(monkeypatch):
    _patch_setup(monkeypatch, lambda s: setattr(s, "lam", np.conj(s.lam)))
    assert _fails(P.test_precond_apply_equals_scan_form, 8, 1e-2)


def test_lambda_modulus_alpha_not_root(monkeypatch):
    _patch_setup(monkeypatch, lambda s: setattr(
        s, "lam", s.lam / np.abs(s.lam) * s.alpha))
    assert _fails(P.test_linear_iterates_closed_form, 1, 16, 8, 1e-2, 1.0,
                  0.0)


def test_phi1_replaced_by_one(monkeypatch):
    _patch_setup(monkeypatch, lambda s: setattr(
        s, "w1", s.dt * np.ones_like(s.w1)))
    assert _fails(P.test_linear_reaction_closed_form, 1)


def test_phi2_term_dropped(monkeypatch):
    _patch_setup(monkeypatch, lambda s: setattr(s, "w2",
                                                np.zeros_like(s.w2)))
    assert _fails(P.test_convergence_order, 2, 2.0)


def test_residual_off_by_one(monkeypatch):
    def bad_shift(st, U, u_first):
        return U.copy()
    monkeypatch.setattr(OE, "_shift", bad_shift)
    assert _fails(P.test_residual_equals_dense_f_minus_QU)


def test_symbol_sign(monkeypatch):
    def flip(s):
        s.mu = -s.mu
        s.E = np.exp(s.dt * s.mu)
    _patch_setup(monkeypatch, flip)
    assert _fails(P.test_symbol_is_laplacian_on_trig_polynomials)
    assert _fails(P.test_single_mode_heat_exact)


def test_nonlinear_derivative_wrong(monkeypatch):
    monkeypatch.setattr(OE.Setup, "dN",
                        lambda self, u: self.n1 + 3.0 * self.n3 * u)
    assert _fails(P.test_nonlinear_sequential_equals_dense_newton, 1, 1, 8,
                  6) is False  # sequential does not use N'
    # Newton-GMRES with a wrong Jacobian still converges (slower) to the
    # unique solution, so the pin is on the Newton step count
    assert _fails(P.test_newton_gmres_reaches_sequential, 1)


# ---------------------------------------------------------------------------
# EBDF2 (Sec. 4)
# ---------------------------------------------------------------------------
import tests.test_oracle_ebdf2 as P2  # noqa: E402


def _patch_both(monkeypatch, name, fn):
    """Replace an oracle function in its module and in the package
    namespace the pins call it through."""
    monkeypatch.setattr(OE, name, fn)
    monkeypatch.setattr(P2.O, name, fn)


def test_ebdf2_lambda1_replaced_by_lambda0(monkeypatch):
    orig = OE.ebdf2_tables

    def bad(st):
        g, l0, l1 = orig(st)
        return g, l0, l0
    _patch_both(monkeypatch, "ebdf2_tables", bad)
    assert _fails(P2.test_ebdf2_precond_equals_dense_inverse, 1, 12, 8, 1e-2)
    assert _fails(P2.test_ebdf2_alpha_circulants_share_eigenvectors, 8, 1e-2)


def test_ebdf2_B_is_A_not_A_squared(monkeypatch):
    monkeypatch.setattr(OE, "_B", lambda st, v: st.A(v))
    assert _fails(P2.test_ebdf2_single_mode_heat_exact)
    assert _fails(P2.test_ebdf2_residual_and_operators_equal_dense)


def test_ebdf2_f2_from_slice_one(monkeypatch):
    def bad_residual(st, u0, U):
        R = np.empty_like(U)
        R[0] = st.A(u0) - U[0]
        f2 = np.zeros_like(U[1:])
        f2[0] = 4.0 / 3.0 * st.A(U[0]) - 1.0 / 3.0 * OE._B(st, u0)
        f2[1] = -1.0 / 3.0 * OE._B(st, U[0])
        R[1:] = f2 - OE.r_apply_ebdf2(st, U[1:])
        return R
    _patch_both(monkeypatch, "residual_ebdf2", bad_residual)
    assert _fails(P2.test_ebdf2_residual_and_operators_equal_dense)


def test_ebdf2_C1_alpha_misplaced(monkeypatch):
    orig = OE.dense_operators_ebdf2

    def bad(st):
        D = orig(st)
        N = st.Nt - 1
        C1a = D["C1"].copy()
        C1a[0, N - 1] = st.alpha        # one column off
        C1a[1, N - 1] = st.alpha
        D["C1a"] = C1a
        I = np.eye(D["R"].shape[0])
        D["Ra"] = I - 4.0 / 3.0 * np.kron(D["C0a"], D["A"]) + \
            1.0 / 3.0 * np.kron(C1a, D["B"])
        return D
    _patch_both(monkeypatch, "dense_operators_ebdf2", bad)
    assert _fails(P2.test_ebdf2_iteration_matrix_spectrum, 6, 0.05, 0.0)


# ---------------------------------------------------------------------------
# complex symbols (advection)
# ---------------------------------------------------------------------------
import tests.test_oracle_complex as PC  # noqa: E402


def test_advection_sign_flipped(monkeypatch):
    def flip(s):
        if any(s.b):
            s.mu = s.mu.real - 1j * s.mu.imag
            s.E = np.exp(s.dt * s.mu)
    _patch_setup(monkeypatch, flip)
    assert _fails(PC.test_advection_diffusion_exact_solution_1d)


def test_advection_nyquist_derivative_kept(monkeypatch):
    def keep(s):
        if any(s.b):
            k = np.fft.fftfreq(s.n, 1.0 / s.n)
            grids = np.meshgrid(*([k] * s.dim), indexing="ij")
            s.mu = -s.a * sum(g * g for g in grids) - s.c - 1j * sum(
                s.b[j] * grids[j] for j in range(s.dim))
            s.E = np.exp(s.dt * s.mu)
    _patch_setup(monkeypatch, keep)
    assert _fails(PC.test_complex_symbol_is_hermitian)


# ---------------------------------------------------------------------------
# IF1 (Sec. 5)
# ---------------------------------------------------------------------------
import tests.test_oracle_if1 as PI  # noqa: E402


def test_if1_nonlinearity_lagged_a_slice(monkeypatch):
    def explicit(st, u0):
        U = np.empty((st.Nt,) + u0.shape)
        prev = u0
        for n in range(st.Nt):
            U[n] = st.A(prev) + st.dt * st.N(prev)
            prev = U[n]
        return U
    monkeypatch.setattr(OE, "sequential_if1", explicit)
    monkeypatch.setattr(PI.O, "sequential_if1", explicit)
    assert _fails(PI.test_if1_sequential_equals_dense_newton, 1, 8, 6, 0.0)


def test_if1_sigma_sign_flipped(monkeypatch):
    orig = OE.precond_apply_if1
    monkeypatch.setattr(OE, "precond_apply_if1",
                        lambda st, R, sigma: orig(st, R, -sigma))
    assert _fails(PI.test_if1_linear_reaction_iterates_closed_form, 1)


# ---------------------------------------------------------------------------
# EBDF3..6 (Sec. bdfs) and BiCGStab
# ---------------------------------------------------------------------------
import tests.test_oracle_ebdf_bicgstab as PS  # noqa: E402


def _patch_pkg(monkeypatch, name, fn):
    monkeypatch.setattr(OE, name, fn)
    monkeypatch.setattr(PS.O, name, fn)


def test_ebdfs_eigenvalue_powers_dropped(monkeypatch):
    orig = OE.ebdf_tables

    def bad(st, s):
        g, lams = orig(st, s)
        return g, [lams[0]] * s
    _patch_pkg(monkeypatch, "ebdf_tables", bad)
    assert _fails(PS.test_precond_is_dense_solve, 4, 0.5)
    assert _fails(PS.test_alpha_circulants_are_powers, 3)


def test_ebdfs_last_coefficient_dropped(monkeypatch):
    orig = OE.ebdf_beta
    _patch_pkg(monkeypatch, "ebdf_beta", lambda s: orig(s)[:-1] + [0.0])
    assert _fails(PS.test_sequential_is_exact_on_linear_problem, 5, 1)
    assert _fails(PS.test_coefficients_are_the_bdf_coefficients, 5)


def test_ebdfs_power_off_by_one(monkeypatch):
    orig = OE._Apow
    monkeypatch.setattr(OE, "_Apow", lambda st, v, j: orig(st, v, j + 1))
    assert _fails(PS.test_sequential_is_exact_on_linear_problem, 3, 1)


def test_ebdfs_fs_from_stored_start_slices(monkeypatch):
    orig = OE._ebdf_start

    def residual_from_U(st, u0, U, s=None):
        s = s or OE.ebdf_order(st.scheme)
        beta = OE.ebdf_beta(s)
        start = orig(st, u0, s)
        R = np.empty_like(U)
        for j in range(1, s):
            R[j - 1] = start[j] - U[j - 1]
        for n in range(s, st.Nt + 1):
            acc = np.zeros_like(U[0])
            for j in range(1, s + 1):
                m = n - j
                w = U[m - 1] if m >= 1 else u0
                acc = acc + beta[j - 1] * OE._Apow(st, w, j)
            R[n - 1] = acc - U[n - 1]
        return R
    _patch_pkg(monkeypatch, "residual_ebdf", residual_from_U)
    assert _fails(PS.test_residual_and_operators_match_dense, 4, 1)


def test_ebdfs_alpha_one_column_off(monkeypatch):
    orig = OE.r_apply_ebdf

    def bad(st, V, s=None):
        s = s or OE.ebdf_order(st.scheme)
        beta = OE.ebdf_beta(s)
        N = V.shape[0]
        out = orig(st, V, s)
        for j in range(1, s + 1):
            for i in range(min(j, N)):
                out[i] -= beta[j - 1] * st.alpha * OE._Apow(
                    st, V[N - j + i - 1], j)
        return out
    _patch_pkg(monkeypatch, "ralpha_apply_ebdf", bad)
    assert _fails(PS.test_residual_and_operators_match_dense, 3, 1)


def test_bicgstab_omega_sign_flipped(monkeypatch):
    src = OE.bicgstab

    def bad(matvec, b, x0, tol=1e-10, max_iter=200):
        # BiCGStab with the stabilising step taken backwards
        x = x0.copy()
        r = b - matvec(x)
        rhat = r.copy()
        p = r.copy()
        rho = np.vdot(rhat, r).real
        it = 0
        while it < max_iter:
            v = matvec(p)
            al = rho / np.vdot(rhat, v).real
            s = r - al * v
            t = matvec(s)
            om = -np.vdot(t, s).real / np.vdot(t, t).real
            x = x + al * p + om * s
            r = s - om * t
            it += 1
            rho_new = np.vdot(rhat, r).real
            p = r + (rho_new / rho) * (al / om) * (p - om * v)
            rho = rho_new
        return x, it, []
    assert src is not bad
    _patch_pkg(monkeypatch, "bicgstab", bad)
    assert _fails(PS.test_bicgstab_iterates_match_scipy, 2)


# ---------------------------------------------------------------------------
# G'(U) and the error metric
# ---------------------------------------------------------------------------
def _patch_oracle(monkeypatch, name, fn):
    """Replace an oracle function in its module and in the package
    namespace the pins call it through."""
    monkeypatch.setattr(OE, name, fn)
    monkeypatch.setattr(P.O, name, fn)


def test_gprime_phi2_terms_dropped(monkeypatch):
    """ETD2's Jacobian without its W2 (J1 - J2) terms: Newton still reaches
    the unique solution, so only the difference pin can see it."""
    orig = OE.gprime_apply

    def bad(st, u0, U, V):
        if st.scheme == 2:
            P1 = OE._shift(st, U, u0)
            V1 = OE._shift(st, V, np.zeros_like(u0))
            return st.W1(st.dN(P1) * V1)
        return orig(st, u0, U, V)
    _patch_oracle(monkeypatch, "gprime_apply", bad)
    assert _fails(P.test_gprime_equals_richardson_difference, 2, 1, 16, 6)
    assert _fails(P.test_gprime_linear_reaction_is_scaled_shift)
    assert not _fails(P.test_gprime_equals_richardson_difference, 1, 1, 16,
                      6)


def test_gprime_unshifted_direction(monkeypatch):
    """N' at u_{n-1} applied to v_n instead of v_{n-1}."""
    def bad(st, u0, U, V):
        P1 = OE._shift(st, U, u0)
        return st.W1(st.dN(P1) * V)
    _patch_oracle(monkeypatch, "gprime_apply", bad)
    assert _fails(P.test_gprime_equals_richardson_difference, 1, 2, 8, 5)


def test_gprime_second_lag_sign(monkeypatch):
    """ETD2's lagged term added instead of subtracted."""
    def bad(st, u0, U, V):
        P1 = OE._shift(st, U, u0)
        V1 = OE._shift(st, V, np.zeros_like(u0))
        P2 = OE._shift(st, P1, u0)
        V2 = OE._shift(st, V1, np.zeros_like(u0))
        J1, J2 = st.dN(P1) * V1, st.dN(P2) * V2
        return st.W1(J1) + st.W2(J1 + J2)
    _patch_oracle(monkeypatch, "gprime_apply", bad)
    assert _fails(P.test_gprime_equals_richardson_difference, 2, 2, 8, 5)


def test_nonlinear_derivative_caught_by_difference_pin(monkeypatch):
    """A wrong N' (the u^2 coefficient dropped) fails the difference pin
    directly, not only through a Newton step count."""
    monkeypatch.setattr(OE.Setup, "dN",
                        lambda self, u: self.n1 + 3.0 * self.n3 * u * u)
    assert _fails(P.test_gprime_equals_richardson_difference, 1, 1, 16, 6)


@pytest.mark.parametrize("bad", [
    lambda U, V: np.linalg.norm(U - V) / np.linalg.norm(V),
    lambda U, V: np.abs(U - V).max() / np.abs(V).max(),
    lambda U, V: (np.sqrt((np.abs(U - V) ** 2).sum(axis=tuple(
        range(1, U.ndim)))).mean()
        / np.sqrt((np.abs(V) ** 2).sum(axis=tuple(range(1, U.ndim)))).mean()),
    lambda U, V: (np.sqrt((np.abs(U - V) ** 2).sum(axis=tuple(
        range(1, U.ndim)))).max()
        / np.sqrt((np.abs(U) ** 2).sum(axis=tuple(range(1, U.ndim)))).max()),
])
def test_rel_err_wrong_norm(monkeypatch, bad):
    _patch_oracle(monkeypatch, "rel_err", bad)
    assert _fails(P.test_rel_err_hand_computed)
