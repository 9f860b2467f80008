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
