"""Thin ctypes binding of libexpdiag.so (include/expdiag.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Device arrays are torch tensors (float64, contiguous, on a HIP device); the
stream is torch's current stream unless one is given.  The library must
have been built (``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

LIB_NAME = "libexpdiag.so"
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), LIB_NAME)

EXPDIAG_OK = 0
EXPDIAG_NOT_CONVERGED = 1
EXPDIAG_EINVAL = -1
EXPDIAG_ENOMEM = -2
EXPDIAG_EHIP = -3
EXPDIAG_EDIVERGED = -4
EXPDIAG_EUNSUPPORTED = -5
EXPDIAG_ETD1 = 1
EXPDIAG_ETD2 = 2
EXPDIAG_EBDF2 = 3
EXPDIAG_IF1 = 4
EXPDIAG_EBDF3 = 5
EXPDIAG_EBDF4 = 6
EXPDIAG_EBDF5 = 7
EXPDIAG_EBDF6 = 8
EXPDIAG_FP64 = 0
EXPDIAG_MIXED = 1

EXPORTED = (
    "expdiag_create", "expdiag_destroy", "expdiag_set_stream",
    "expdiag_footprint_bytes", "expdiag_residual", "expdiag_precond_apply",
    "expdiag_iterate", "expdiag_gmres", "expdiag_bicgstab",
    "expdiag_newton_apply",
    "expdiag_profile_enable",
    "expdiag_profile_read", "expdiag_strerror", "expdiag_last_error",
    "expdiag_set_graph", "expdiag_batch_create", "expdiag_batch_destroy",
    "expdiag_batch_iterate", "expdiag_batch_iterate_each",
    "expdiag_batch_last_error",
    "expdiag_server_create", "expdiag_server_submit", "expdiag_server_poll",
    "expdiag_server_stats", "expdiag_server_destroy",
    "expdiag_set_time_variant", "expdiag_get_time_variant",
    "expdiag_autotune", "expdiag_iterate_noalloc", "expdiag_get_tuning",
    "expdiag_set_tuning",
    "expdiag_batch_autotune", "expdiag_batch_graph",
    "expdiag_server_autotune", "expdiag_set_zero_guess",
    "expdiag_batch_set_zero_guess",
)


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3)]


class Problem(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("c", ctypes.c_double),
                ("n1", ctypes.c_double), ("n2", ctypes.c_double),
                ("n3", ctypes.c_double), ("precision", ctypes.c_int),
                ("gmres_restart", ctypes.c_int),
                ("b", ctypes.c_double * 3),
                ("a_im", ctypes.c_double), ("c_im", ctypes.c_double),
                ("complex_state", ctypes.c_int), ("jacobian", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_longlong), ("status", ctypes.c_int),
                ("iters", ctypes.c_int), ("rel_update", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ExpdiagError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"expdiag error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with __graft_entry__.build(); "
            "there is no CPU fallback")
    L = ctypes.CDLL(path)
    vp, cd, ci, sz = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, \
        ctypes.c_size_t
    L.expdiag_create.argtypes = [ctypes.POINTER(Grid), ci, cd, cd, ci,
                                 ctypes.POINTER(Problem), vp,
                                 ctypes.POINTER(vp)]
    L.expdiag_destroy.argtypes = [vp]
    L.expdiag_set_stream.argtypes = [vp, vp]
    L.expdiag_footprint_bytes.argtypes = [ctypes.POINTER(Grid), ci, ci, ci,
                                          ci]
    L.expdiag_footprint_bytes.restype = sz
    L.expdiag_residual.argtypes = [vp, vp, vp, vp,
                                   ctypes.POINTER(cd)]
    L.expdiag_precond_apply.argtypes = [vp, vp, vp]
    L.expdiag_iterate.argtypes = [vp, vp, vp, ci, cd,
                                  ctypes.POINTER(ci), ctypes.POINTER(cd)]
    L.expdiag_gmres.argtypes = [vp, vp, vp, ci, ci, cd,
                                ctypes.POINTER(ci), ctypes.POINTER(cd)]
    L.expdiag_bicgstab.argtypes = [vp, vp, vp, ci, cd,
                                   ctypes.POINTER(ci), ctypes.POINTER(cd)]
    L.expdiag_newton_apply.argtypes = [vp, vp, vp, vp, vp]
    L.expdiag_profile_enable.argtypes = [vp, ci]
    L.expdiag_profile_read.argtypes = [vp, ctypes.POINTER(cd),
                                       ctypes.POINTER(ctypes.c_long),
                                       ctypes.POINTER(cd),
                                       ctypes.POINTER(ctypes.c_long), ci]
    L.expdiag_set_graph.argtypes = [vp, ci]
    L.expdiag_set_zero_guess.argtypes = [vp, ci]
    L.expdiag_batch_set_zero_guess.argtypes = [vp, ci]
    L.expdiag_set_time_variant.argtypes = [vp, ci]
    L.expdiag_get_time_variant.argtypes = [vp]
    L.expdiag_autotune.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ci),
                                   ctypes.POINTER(cd), ctypes.POINTER(cd)]
    L.expdiag_get_tuning.argtypes = [vp, ctypes.POINTER(ci),
                                     ctypes.POINTER(ci)]
    L.expdiag_set_tuning.argtypes = [vp, ci, ci]
    pp = ctypes.POINTER(vp)
    L.expdiag_batch_autotune.argtypes = [vp, pp, pp, ctypes.c_char_p,
                                         ctypes.POINTER(ci),
                                         ctypes.POINTER(ci),
                                         ctypes.POINTER(cd),
                                         ctypes.POINTER(cd)]
    L.expdiag_batch_graph.argtypes = [vp]
    L.expdiag_batch_create.argtypes = [pp, ci, vp, pp]
    L.expdiag_batch_destroy.argtypes = [vp]
    L.expdiag_batch_iterate.argtypes = [vp, pp, pp, ci, cd,
                                        ctypes.POINTER(ci),
                                        ctypes.POINTER(cd),
                                        ctypes.POINTER(ci)]
    L.expdiag_batch_iterate_each.argtypes = [vp, pp, pp,
                                             ctypes.POINTER(ci),
                                             ctypes.POINTER(cd),
                                             ctypes.POINTER(ci),
                                             ctypes.POINTER(cd),
                                             ctypes.POINTER(ci)]
    L.expdiag_batch_last_error.argtypes = [vp]
    L.expdiag_batch_last_error.restype = ctypes.c_char_p
    L.expdiag_server_create.argtypes = [sz, ci, vp, pp]
    L.expdiag_server_submit.argtypes = [vp, ctypes.POINTER(Grid), ci, cd, cd,
                                        ci, ctypes.POINTER(Problem), vp, vp,
                                        ci, cd,
                                        ctypes.POINTER(ctypes.c_longlong)]
    L.expdiag_server_poll.argtypes = [vp, ctypes.POINTER(Result), ci,
                                      ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.expdiag_server_stats.argtypes = [vp, ctypes.POINTER(sz),
                                       ctypes.POINTER(ci),
                                       ctypes.POINTER(ci),
                                       ctypes.POINTER(cd)]
    L.expdiag_server_destroy.argtypes = [vp]
    L.expdiag_server_autotune.argtypes = [vp, ctypes.c_char_p]
    L.expdiag_iterate_noalloc.argtypes = [ctypes.POINTER(Grid), ci, cd, cd,
                                          ci, ctypes.POINTER(Problem), vp,
                                          vp, vp, ci, cd, ctypes.POINTER(ci),
                                          ctypes.POINTER(cd)]
    L.expdiag_strerror.argtypes = [ci]
    L.expdiag_strerror.restype = ctypes.c_char_p
    L.expdiag_last_error.argtypes = [vp]
    L.expdiag_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        getattr(L, name).restype = getattr(L, name).restype or ci
    _lib = L
    return L


def make_grid(shape: Sequence[int]) -> Grid:
    g = Grid()
    g.dim = len(shape)
    for i in range(3):
        g.n[i] = int(shape[i]) if i < len(shape) else 1
    return g


def make_problem(a, c=0.0, n1=0.0, n2=0.0, n3=0.0, precision=EXPDIAG_FP64,
                 gmres_restart=0, b=(0.0, 0.0, 0.0), a_im=0.0, c_im=0.0,
                 complex_state=None, jacobian=1) -> Problem:
    """complex_state defaults to 1 when a_im or c_im is nonzero; jacobian
    (IF1 only): 0 none, 1 mean N'(U^k), 2 mean N'(u0)."""
    bb = tuple(float(v) for v in b) + (0.0,) * (3 - len(b))
    if complex_state is None:
        complex_state = 1 if (a_im != 0.0 or c_im != 0.0) else 0
    return Problem(float(a), float(c), float(n1), float(n2), float(n3),
                   int(precision), int(gmres_restart),
                   (ctypes.c_double * 3)(*bb[:3]), float(a_im), float(c_im),
                   int(complex_state), int(jacobian))


def _ptr(t, numel=None, name="array"):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype not in (torch.float64, torch.complex128) or \
            not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name} must be a contiguous float64 or "
                         "complex128 GPU tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def strerror(code: int) -> str:
    return load().expdiag_strerror(code).decode()


def _check(rc, h=None, ok=(EXPDIAG_OK,)):
    if rc in ok:
        return rc
    L = load()
    msg = L.expdiag_last_error(h).decode() if h is not None else \
        L.expdiag_last_error(None).decode()
    raise ExpdiagError(rc, f"{strerror(rc)}: {msg}")


# -- the C ABI, one Python function per entry point ------------------------
def expdiag_create(shape, Nt, dt, alpha, scheme, problem: Problem,
                   stream=None):
    L = load()
    h = ctypes.c_void_p()
    g = make_grid(shape)
    rc = L.expdiag_create(ctypes.byref(g), int(Nt), float(dt), float(alpha),
                          int(scheme), ctypes.byref(problem),
                          _stream(stream), ctypes.byref(h))
    _check(rc)
    return h


def expdiag_destroy(h):
    return load().expdiag_destroy(h)


def expdiag_set_stream(h, stream):
    return _check(load().expdiag_set_stream(h, _stream(stream)), h)


def expdiag_footprint_bytes(shape, Nt, scheme, precision=EXPDIAG_FP64,
                            gmres_restart=0) -> int:
    g = make_grid(shape)
    return int(load().expdiag_footprint_bytes(ctypes.byref(g), int(Nt),
                                              int(scheme), int(precision),
                                              int(gmres_restart)))


def expdiag_residual(h, u0, U, R, want_norm=True):
    nrm = ctypes.c_double(0.0)
    rc = load().expdiag_residual(h, _ptr(u0, name="u0"), _ptr(U, name="U"),
                                 _ptr(R, U.numel(), "R"),
                                 ctypes.byref(nrm) if want_norm else None)
    _check(rc, h)
    return nrm.value if want_norm else None


def expdiag_precond_apply(h, R, S):
    return _check(load().expdiag_precond_apply(
        h, _ptr(R, name="R"), _ptr(S, R.numel(), "S")), h)


def expdiag_iterate(h, u0, U, max_iter, tol):
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = load().expdiag_iterate(h, _ptr(u0, name="u0"), _ptr(U, name="U"),
                                int(max_iter), float(tol), ctypes.byref(it),
                                ctypes.byref(rel))
    _check(rc, h, ok=(EXPDIAG_OK, EXPDIAG_NOT_CONVERGED))
    return rc, it.value, rel.value


def expdiag_gmres(h, u0, U, restart, max_iter, tol):
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = load().expdiag_gmres(h, _ptr(u0, name="u0"), _ptr(U, name="U"),
                              int(restart), int(max_iter), float(tol),
                              ctypes.byref(it), ctypes.byref(rel))
    _check(rc, h, ok=(EXPDIAG_OK, EXPDIAG_NOT_CONVERGED))
    return rc, it.value, rel.value


def expdiag_bicgstab(h, u0, U, max_iter, tol):
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = load().expdiag_bicgstab(h, _ptr(u0, name="u0"), _ptr(U, name="U"),
                                 int(max_iter), float(tol), ctypes.byref(it),
                                 ctypes.byref(rel))
    _check(rc, h, ok=(EXPDIAG_OK, EXPDIAG_NOT_CONVERGED))
    return rc, it.value, rel.value


def expdiag_newton_apply(h, u0, U, V, W):
    n = U.numel()
    return _check(load().expdiag_newton_apply(
        h, _ptr(u0, name="u0"), _ptr(U, name="U"), _ptr(V, n, "V"),
        _ptr(W, n, "W")), h)


def expdiag_iterate_noalloc(shape, Nt, dt, alpha, scheme, problem: Problem,
                            u0, U, max_iter, tol, stream=None):
    """The solve of create + iterate + destroy with no device allocation
    (the library's fixed workspace); returns (rc, iters, rel_update)."""
    L = load()
    g = make_grid(shape)
    ns = 1
    for v in shape:
        ns *= int(v)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = L.expdiag_iterate_noalloc(ctypes.byref(g), int(Nt), float(dt),
                                   float(alpha), int(scheme),
                                   ctypes.byref(problem), _stream(stream),
                                   _ptr(u0, name="u0"),
                                   _ptr(U, int(Nt) * ns, "U"), int(max_iter),
                                   float(tol), ctypes.byref(it),
                                   ctypes.byref(rel))
    _check(rc, None, ok=(EXPDIAG_OK, EXPDIAG_NOT_CONVERGED))
    return rc, it.value, rel.value


def expdiag_profile_enable(h, mask=0x1F):
    """mask: bit i brackets launches of class i with events; 0 disables."""
    return _check(load().expdiag_profile_enable(h, int(mask)), h)


PROFILE_CLASSES = ("col_fft", "row_fft", "passb", "reduce", "krylov")


def expdiag_profile_read(h, nclass=5):
    """Returns (ms, launches, bytes, timed_launches) per kernel class."""
    ms = (ctypes.c_double * nclass)()
    cnt = (ctypes.c_long * nclass)()
    by = (ctypes.c_double * nclass)()
    tm = (ctypes.c_long * nclass)()
    _check(load().expdiag_profile_read(h, ms, cnt, by, tm, nclass), h)
    return list(ms), list(cnt), list(by), list(tm)


class Solver:
    """Owns one handle; convenience wrapper around the functions above."""

    def __init__(self, shape, Nt, dt, alpha, scheme=EXPDIAG_ETD1, a=1.0,
                 c=0.0, n1=0.0, n2=0.0, n3=0.0, precision=EXPDIAG_FP64,
                 gmres_restart=0, stream=None, b=(0.0, 0.0, 0.0), a_im=0.0,
                 c_im=0.0, complex_state=None, jacobian=1):
        self.shape = tuple(int(v) for v in shape)
        self.Nt = int(Nt)
        self.problem = make_problem(a, c, n1, n2, n3, precision,
                                    gmres_restart, b, a_im, c_im,
                                    complex_state, jacobian)
        self.h = expdiag_create(self.shape, Nt, dt, alpha, scheme,
                                self.problem, stream)

    @classmethod
    def from_instance(cls, inst, gmres_restart=0, stream=None,
                      precision=None):
        return cls(inst.shape, inst.Nt, inst.dt, inst.alpha, inst.scheme,
                   inst.a, inst.c, inst.n1, inst.n2, inst.n3,
                   inst.precision if precision is None else precision,
                   gmres_restart, stream, getattr(inst, "b", (0.0, 0.0, 0.0)),
                   getattr(inst, "a_im", 0.0), getattr(inst, "c_im", 0.0),
                   1 if getattr(inst, "cstate", False) else None,
                   getattr(inst, "jac", 1))

    def close(self):
        if self.h is not None:
            expdiag_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def residual(self, u0, U, R):
        return expdiag_residual(self.h, u0, U, R)

    def precond_apply(self, R, S):
        return expdiag_precond_apply(self.h, R, S)

    def iterate(self, u0, U, max_iter=200, tol=1e-11):
        return expdiag_iterate(self.h, u0, U, max_iter, tol)

    def set_zero_guess(self, on=True):
        return expdiag_set_zero_guess(self.h, on)

    def gmres(self, u0, U, restart=20, max_iter=400, tol=1e-10):
        return expdiag_gmres(self.h, u0, U, restart, max_iter, tol)

    def bicgstab(self, u0, U, max_iter=400, tol=1e-10):
        return expdiag_bicgstab(self.h, u0, U, max_iter, tol)

    def newton_apply(self, u0, U, V, W):
        return expdiag_newton_apply(self.h, u0, U, V, W)


def expdiag_set_graph(h, on=True):
    return _check(load().expdiag_set_graph(h, 1 if on else 0), h)


def expdiag_set_zero_guess(h, on=True):
    return _check(load().expdiag_set_zero_guess(h, 1 if on else 0), h)


# -- batching -----------------------------------------------------------------
def expdiag_batch_create(handles, stream=None):
    L = load()
    arr = (ctypes.c_void_p * len(handles))(*[h.value for h in handles])
    b = ctypes.c_void_p()
    rc = L.expdiag_batch_create(arr, len(handles), _stream(stream),
                                ctypes.byref(b))
    _check(rc)
    return b


def expdiag_batch_destroy(b):
    return load().expdiag_batch_destroy(b)


def expdiag_batch_iterate(b, u0s, Us, max_iter, tol):
    """Returns (rc, iters[], rel_update[], status[])."""
    L = load()
    n = len(u0s)
    if len(Us) != n:
        raise ValueError("u0s and Us differ in length")
    pu = (ctypes.c_void_p * n)(*[_ptr(t, name="u0").value for t in u0s])
    pU = (ctypes.c_void_p * n)(*[_ptr(t, name="U").value for t in Us])
    it = (ctypes.c_int * n)()
    rel = (ctypes.c_double * n)()
    st = (ctypes.c_int * n)()
    rc = L.expdiag_batch_iterate(b, pu, pU, int(max_iter), float(tol), it,
                                 rel, st)
    if rc < 0 and rc != EXPDIAG_EDIVERGED:
        raise ExpdiagError(rc, f"{strerror(rc)}: "
                           f"{L.expdiag_batch_last_error(b).decode()}")
    return rc, list(it), list(rel), list(st)


def expdiag_batch_iterate_each(b, u0s, Us, max_iters, tols):
    """Per-instance caps and tolerances; returns (rc, iters[],
    rel_update[], status[])."""
    L = load()
    n = len(u0s)
    if len(Us) != n or len(max_iters) != n or len(tols) != n:
        raise ValueError("u0s, Us, max_iters and tols differ in length")
    pu = (ctypes.c_void_p * n)(*[_ptr(t, name="u0").value for t in u0s])
    pU = (ctypes.c_void_p * n)(*[_ptr(t, name="U").value for t in Us])
    caps = (ctypes.c_int * n)(*[int(v) for v in max_iters])
    tl = (ctypes.c_double * n)(*[float(v) for v in tols])
    it = (ctypes.c_int * n)()
    rel = (ctypes.c_double * n)()
    st = (ctypes.c_int * n)()
    rc = L.expdiag_batch_iterate_each(b, pu, pU, caps, tl, it, rel, st)
    if rc < 0 and rc != EXPDIAG_EDIVERGED:
        raise ExpdiagError(rc, f"{strerror(rc)}: "
                           f"{L.expdiag_batch_last_error(b).decode()}")
    return rc, list(it), list(rel), list(st)


def expdiag_batch_autotune(b, u0s, Us, cache_path=None):
    """Returns dict(shapes, graph_used, ms_graph, ms_launch)."""
    L = load()
    n = len(u0s)
    pu = (ctypes.c_void_p * n)(*[_ptr(t, name="u0").value for t in u0s])
    pU = (ctypes.c_void_p * n)(*[_ptr(t, name="U").value for t in Us])
    sh, gu = ctypes.c_int(0), ctypes.c_int(0)
    mg, ml = ctypes.c_double(0.0), ctypes.c_double(0.0)
    path = None if cache_path is None else str(cache_path).encode()
    rc = L.expdiag_batch_autotune(b, pu, pU, path, ctypes.byref(sh),
                                  ctypes.byref(gu), ctypes.byref(mg),
                                  ctypes.byref(ml))
    if rc != EXPDIAG_OK:
        raise ExpdiagError(rc, f"{strerror(rc)}: "
                           f"{L.expdiag_batch_last_error(b).decode()}")
    return dict(shapes=sh.value, graph_used=bool(gu.value),
                ms_graph=mg.value, ms_launch=ml.value)


def expdiag_batch_graph(b):
    return bool(load().expdiag_batch_graph(b))


def expdiag_batch_set_zero_guess(b, on=True):
    rc = load().expdiag_batch_set_zero_guess(b, 1 if on else 0)
    if rc != EXPDIAG_OK:
        raise ExpdiagError(rc, strerror(rc))
    return rc


class Batch:
    """Owns a batch over existing Solvers (which stay owned by the caller)."""

    def __init__(self, solvers, stream=None):
        self.solvers = list(solvers)
        self.b = expdiag_batch_create([s.h for s in self.solvers], stream)

    def iterate(self, u0s, Us, max_iter=400, tol=1e-11):
        return expdiag_batch_iterate(self.b, u0s, Us, max_iter, tol)

    def iterate_each(self, u0s, Us, max_iters, tols):
        return expdiag_batch_iterate_each(self.b, u0s, Us, max_iters, tols)

    def autotune(self, u0s, Us, cache_path=None):
        return expdiag_batch_autotune(self.b, u0s, Us, cache_path)

    def set_zero_guess(self, on=True):
        return expdiag_batch_set_zero_guess(self.b, on)

    def close(self):
        if self.b is not None:
            expdiag_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- serving ------------------------------------------------------------------
def expdiag_server_create(hbm_budget, max_active, stream=None):
    s = ctypes.c_void_p()
    _check(load().expdiag_server_create(int(hbm_budget), int(max_active),
                                        _stream(stream), ctypes.byref(s)))
    return s


def expdiag_server_submit(s, shape, Nt, dt, alpha, scheme, problem, u0, U,
                          max_iter, tol):
    rid = ctypes.c_longlong(0)
    g = make_grid(shape)
    rc = load().expdiag_server_submit(s, ctypes.byref(g), int(Nt), float(dt),
                                      float(alpha), int(scheme),
                                      ctypes.byref(problem),
                                      _ptr(u0, name="u0"), _ptr(U, name="U"),
                                      int(max_iter), float(tol),
                                      ctypes.byref(rid))
    _check(rc)
    return rid.value


def expdiag_server_poll(s, cap=256):
    out = (Result * cap)()
    n = ctypes.c_int(0)
    pending = ctypes.c_int(0)
    _check(load().expdiag_server_poll(s, out, cap, ctypes.byref(n),
                                      ctypes.byref(pending)))
    res = [dict(id=r.id, status=r.status, iters=r.iters,
                rel_update=r.rel_update, t_submit=r.t_submit,
                t_admit=r.t_admit, t_done=r.t_done) for r in out[:n.value]]
    return res, pending.value


def expdiag_server_stats(s):
    b = ctypes.c_size_t(0)
    a = ctypes.c_int(0)
    p = ctypes.c_int(0)
    busy = ctypes.c_double(0.0)
    _check(load().expdiag_server_stats(s, ctypes.byref(b), ctypes.byref(a),
                                       ctypes.byref(p), ctypes.byref(busy)))
    return dict(bytes_in_use=b.value, active=a.value, pending=p.value,
                busy_s=busy.value)


def expdiag_server_destroy(s):
    return load().expdiag_server_destroy(s)


# -- time-transform variant and autotuning ---------------------------------
TIME_FFT = 0
TIME_DENSE_MFMA = 1


def expdiag_set_time_variant(h, variant):
    return _check(load().expdiag_set_time_variant(h, int(variant)), h)


def expdiag_get_time_variant(h):
    return load().expdiag_get_time_variant(h)


def expdiag_get_tuning(h):
    """Returns (time_variant, col_wide)."""
    v = ctypes.c_int(0)
    w = ctypes.c_int(0)
    _check(load().expdiag_get_tuning(h, ctypes.byref(v), ctypes.byref(w)), h)
    return v.value, w.value


def expdiag_set_tuning(h, time_variant, col_wide):
    return _check(load().expdiag_set_tuning(h, int(time_variant),
                                            int(col_wide)), h)


def expdiag_server_autotune(s, cache_path=None):
    path = None if cache_path is None else str(cache_path).encode()
    return _check(load().expdiag_server_autotune(s, path))


def expdiag_autotune(h, cache_path=None):
    """Returns (variant, us_fft, us_dense) and applies the variant."""
    v = ctypes.c_int(0)
    a = ctypes.c_double(0.0)
    b = ctypes.c_double(0.0)
    path = None if cache_path is None else str(cache_path).encode()
    _check(load().expdiag_autotune(h, path, ctypes.byref(v), ctypes.byref(a),
                                   ctypes.byref(b)), h)
    return v.value, a.value, b.value
