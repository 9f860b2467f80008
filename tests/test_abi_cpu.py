"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2603_04350_amd import expdiag as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "expdiag.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(expdiag_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(X.LIB_PATH):
        pytest.skip("libexpdiag.so not built")
    return X.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "expdiag_iterate" in names and "expdiag_gmres" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(X.EXPORTED)


def test_strerror(lib):
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert lib.expdiag_strerror(code)
    assert b"unknown" in lib.expdiag_strerror(12345)


def _create(lib, shape, Nt, dt, alpha, scheme, prob):
    h = ctypes.c_void_p()
    g = X.make_grid(shape)
    return lib.expdiag_create(ctypes.byref(g), Nt, dt, alpha, scheme,
                              ctypes.byref(prob), None, ctypes.byref(h)), h


@pytest.mark.parametrize("shape,Nt,dt,alpha,scheme,prob,code", [
    ((63,), 8, 0.1, 1e-2, 1, X.make_problem(1.0), X.EXPDIAG_EINVAL),
    ((2,), 8, 0.1, 1e-2, 1, X.make_problem(1.0), X.EXPDIAG_EINVAL),
    ((96,), 8, 0.1, 1e-2, 1, X.make_problem(1.0), X.EXPDIAG_EUNSUPPORTED),
    ((8192,), 8, 0.1, 1e-2, 1, X.make_problem(1.0), X.EXPDIAG_EUNSUPPORTED),
    ((64,), 1, 0.1, 1e-2, 1, X.make_problem(1.0), X.EXPDIAG_EINVAL),
    ((64,), 12, 0.1, 1e-2, 1, X.make_problem(1.0), X.EXPDIAG_EUNSUPPORTED),
    ((64,), 8, 0.0, 1e-2, 1, X.make_problem(1.0), X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 0.0, 1, X.make_problem(1.0), X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 1.0, 1, X.make_problem(1.0), X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 1e-2, 9, X.make_problem(1.0), X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 1e-2, 0, X.make_problem(1.0), X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 1e-2, X.EXPDIAG_IF1, X.make_problem(1.0, jacobian=3),
     X.EXPDIAG_EINVAL),
    # EBDF2: linear problems, 8 <= Nt <= 128
    ((64,), 8, 0.1, 1e-2, X.EXPDIAG_EBDF2, X.make_problem(1.0, n1=1.0),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 4, 0.1, 1e-2, X.EXPDIAG_EBDF2, X.make_problem(1.0),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 256, 0.1, 1e-2, X.EXPDIAG_EBDF2, X.make_problem(1.0),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 66, 0.1, 1e-2, X.EXPDIAG_EBDF2, X.make_problem(1.0),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 1025, 0.1, 1e-2, X.EXPDIAG_EBDF2, X.make_problem(1.0),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 65, 0.1, 1e-2, X.EXPDIAG_ETD1, X.make_problem(1.0),
     X.EXPDIAG_EUNSUPPORTED),
    # EBDF3..6: linear; Nt - s + 1 a power of two 2..512, or Nt one 8..128
    ((64,), 16, 0.1, 1e-2, X.EXPDIAG_EBDF4, X.make_problem(1.0, n3=-1.0),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 65, 0.1, 1e-2, X.EXPDIAG_EBDF3, X.make_problem(1.0),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 6, 0.1, 1e-2, X.EXPDIAG_EBDF6, X.make_problem(1.0),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 4, 0.1, 1e-2, X.EXPDIAG_EBDF4, X.make_problem(1.0),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 518, 0.1, 1e-2, X.EXPDIAG_EBDF6, X.make_problem(1.0),
     X.EXPDIAG_EUNSUPPORTED),
    # complex coefficients need a complex state; a complex state is linear
    ((64,), 8, 0.1, 1e-2, 1, X.make_problem(0.0, a_im=1.0, complex_state=0),
     X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 1e-2, 1, X.make_problem(1.0, complex_state=2),
     X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 1e-2, 1, X.make_problem(1.0, n1=1.0, complex_state=1),
     X.EXPDIAG_EUNSUPPORTED),
    ((64,), 8, 0.1, 1e-2, 1, X.make_problem(1.0, b=(float("nan"),)),
     X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 1e-2, 1, X.make_problem(-1.0), X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 1e-2, 1, X.make_problem(1.0, c=-0.1), X.EXPDIAG_EINVAL),
    ((64,), 8, 0.1, 1e-2, 1, X.make_problem(1.0, precision=7),
     X.EXPDIAG_EINVAL),
    ((64, 64, 64, 64), 8, 0.1, 1e-2, 1, X.make_problem(1.0),
     X.EXPDIAG_EINVAL),
])
def test_create_rejects_invalid_arguments(lib, shape, Nt, dt, alpha, scheme,
                                          prob, code):
    if len(shape) > 3:
        g = X.Grid()
        g.dim = 4
        h = ctypes.c_void_p()
        rc = lib.expdiag_create(ctypes.byref(g), Nt, dt, alpha, scheme,
                                ctypes.byref(prob), None, ctypes.byref(h))
    else:
        rc, h = _create(lib, shape, Nt, dt, alpha, scheme, prob)
    assert rc == code
    assert h.value is None
    assert lib.expdiag_last_error(None)


def test_null_handle_calls_are_rejected(lib):
    assert lib.expdiag_iterate(None, None, None, 1, 0.0, None, None) == \
        X.EXPDIAG_EINVAL
    assert lib.expdiag_precond_apply(None, None, None) == X.EXPDIAG_EINVAL
    assert lib.expdiag_newton_apply(None, None, None, None, None) == \
        X.EXPDIAG_EINVAL
    assert lib.expdiag_batch_iterate_each(None, None, None, None, None,
                                          None, None, None) == \
        X.EXPDIAG_EINVAL
    assert lib.expdiag_iterate_noalloc(None, 8, 0.1, 1e-2, 1, None, None,
                                       None, None, 10, 0.0, None, None) == \
        X.EXPDIAG_EINVAL
    assert lib.expdiag_set_zero_guess(None, 1) == X.EXPDIAG_EINVAL
    assert lib.expdiag_batch_set_zero_guess(None, 1) == X.EXPDIAG_EINVAL
    assert lib.expdiag_destroy(None) == X.EXPDIAG_OK


def test_footprint_bytes(lib):
    fp = X.expdiag_footprint_bytes((256, 256), 64, 1)
    Nk = 256 * 129
    state = 64 * Nk * 16
    assert 3 * state <= fp <= 3 * state + 8 * 1024 * 1024
    assert X.expdiag_footprint_bytes((63,), 8, 1) == 0
    assert X.expdiag_footprint_bytes((256, 256), 64, 1, gmres_restart=20) > \
        20 * state
    # EBDF2 is linear: no nonlinear buffer; outside 8..128 it is unsupported
    fb = X.expdiag_footprint_bytes((256, 256), 64, X.EXPDIAG_EBDF2)
    assert 2 * state <= fb < 3 * state
    assert X.expdiag_footprint_bytes((256, 256), 256, X.EXPDIAG_EBDF2) == 0
    assert X.expdiag_footprint_bytes((256, 256), 65, X.EXPDIAG_EBDF2) > \
        2 * state
    assert X.expdiag_footprint_bytes((256, 256), 65, X.EXPDIAG_ETD1) == 0
    # EBDF3..6 likewise: Nt - s + 1 a power of two, or Nt one in 8..128
    for sch, Nt_fft in ((X.EXPDIAG_EBDF3, 66), (X.EXPDIAG_EBDF4, 67),
                        (X.EXPDIAG_EBDF5, 68), (X.EXPDIAG_EBDF6, 69)):
        assert 2 * state <= X.expdiag_footprint_bytes(
            (256, 256), 64, sch) < 3 * state
        assert X.expdiag_footprint_bytes((256, 256), Nt_fft, sch) > 2 * state
        assert X.expdiag_footprint_bytes((256, 256), 65, sch) == 0
    assert X.expdiag_footprint_bytes((256, 256), 64, 9) == 0
