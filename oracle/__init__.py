"""Plain FP64 CPU oracle for the atom + trapped-ion ensemble integration.

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It wraps ``libaio.so``,
built from ``aio.c`` (plain C, FP64, no contraction, no fast math) with gcc;
it shares no source with the HIP library and imports nothing from it.

System constants are passed as any object (or mapping) with the attributes
m_ion, m_atom, n, m, Cn, Cm, a, q, omega_rf, r_exit, r_bounce, max_steps, hmax
(atomic units).  Ensembles are (12, n) float64 arrays of planes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaio.so")
SOURCES = [os.path.join(_HERE, "aio.c"), os.path.join(_HERE, "aio.h")]
NSTATE = 12
NOBS = 13
OK, EINVAL, WRTOL = 0, -1, 1

_lock = threading.Lock()
_lib = None


def build() -> str:
    """Compile libaio.so in place with gcc."""
    tmp = LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-Wall",
           "-fPIC", "-shared", "-pthread", "-o", tmp, SOURCES[0], "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _stale() -> bool:
    built = os.path.getmtime(LIB_PATH)
    return any(os.path.getmtime(src) > built for src in SOURCES)


class System(C.Structure):
    _fields_ = [
        ("m_ion", C.c_double), ("m_atom", C.c_double),
        ("n", C.c_int), ("m", C.c_int),
        ("Cn", C.c_double), ("Cm", C.c_double),
        ("a", C.c_double * 3), ("q", C.c_double * 3),
        ("omega_rf", C.c_double), ("r_exit", C.c_double), ("r_bounce", C.c_double),
        ("max_steps", C.c_longlong), ("hmax", C.c_double),
    ]


class Run(C.Structure):
    _fields_ = [
        ("t_end", C.c_double), ("h_next", C.c_double),
        ("nsteps", C.c_longlong), ("nfailed", C.c_longlong), ("nfevals", C.c_longlong),
        ("status", C.c_int), ("rtol_raised", C.c_int),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def _get(obj, name):
    return obj[name] if isinstance(obj, dict) else getattr(obj, name)


def system(obj) -> System:
    s = System()
    s.m_ion = float(_get(obj, "m_ion"))
    s.m_atom = float(_get(obj, "m_atom"))
    s.n = int(_get(obj, "n"))
    s.m = int(_get(obj, "m"))
    s.Cn = float(_get(obj, "Cn"))
    s.Cm = float(_get(obj, "Cm"))
    for k in range(3):
        s.a[k] = float(_get(obj, "a")[k])
        s.q[k] = float(_get(obj, "q")[k])
    s.omega_rf = float(_get(obj, "omega_rf"))
    s.r_exit = float(_get(obj, "r_exit"))
    s.r_bounce = float(_get(obj, "r_bounce"))
    s.max_steps = int(_get(obj, "max_steps"))
    s.hmax = float(_get(obj, "hmax"))
    return s


_D = C.POINTER(C.c_double)
RHS = C.CFUNCTYPE(None, C.c_void_p, C.c_double, _D, _D)


def _wrap_rhs(fun, dim):
    """C callback around fun(t, y) -> dy/dt (numpy arrays of length dim)."""
    def cb(_ctx, t, yp, fp):
        y = np.ctypeslib.as_array(yp, shape=(dim,)).copy()
        out = np.asarray(fun(t, y), dtype=np.float64)
        f = np.ctypeslib.as_array(fp, shape=(dim,))
        f[:] = out
    return RHS(cb)


def load():
    """The oracle library, built first if it is missing."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH) or _stale():
            build()
        lib = C.CDLL(LIB_PATH)
        lib.aio_version.restype = C.c_int
        lib.aio_tableau.argtypes = [_D] * 5
        lib.aio_force.argtypes = [C.POINTER(System), C.c_double, _D, _D]
        lib.aio_energy.argtypes = [C.POINTER(System), C.c_double, _D]
        lib.aio_energy.restype = C.c_double
        lib.aio_spacing.argtypes = [C.c_double]
        lib.aio_spacing.restype = C.c_double
        lib.aio_initial_step.argtypes = [C.c_int, _D, _D, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double]
        lib.aio_initial_step.restype = C.c_double
        lib.aio_error_norm.argtypes = [C.c_int, C.c_double, _D, _D, _D, C.c_double]
        lib.aio_error_norm.restype = C.c_double
        lib.aio_step_after_failure.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int,
                                               C.c_double]
        lib.aio_step_after_failure.restype = C.c_double
        lib.aio_step_after_success.argtypes = [C.c_double, C.c_double, C.c_double]
        lib.aio_step_after_success.restype = C.c_double
        lib.aio_linear_attempt.argtypes = [C.c_int, _D, C.c_double, C.c_double, _D, _D, _D]
        lib.aio_linear_ode45.argtypes = [C.c_int, _D, C.c_double, C.c_double, _D, C.c_double,
                                         C.c_double, C.c_double, C.c_longlong, _D,
                                         C.POINTER(Run), _D, _D, C.c_longlong]
        lib.aio_linear_ode45.restype = C.c_int
        lib.aio_rhs_attempt.argtypes = [C.c_int, RHS, C.c_void_p, C.c_double, C.c_double, _D,
                                        _D, _D]
        lib.aio_rhs_ode45.argtypes = [C.c_int, RHS, C.c_void_p, C.c_double, C.c_double, _D,
                                      C.c_double, C.c_double, C.c_double, C.c_longlong, _D,
                                      C.POINTER(Run), _D, _D, C.c_longlong]
        lib.aio_rhs_ode45.restype = C.c_int
        lib.aio_integrate_one.argtypes = [C.POINTER(System), C.c_double, C.c_double, _D,
                                          C.c_double, C.c_double, _D, _D]
        lib.aio_integrate_one.restype = C.c_int
        lib.aio_integrate.argtypes = [C.POINTER(System), _D, C.c_longlong, C.c_longlong,
                                      C.c_double, C.c_double, C.c_double, C.c_double, _D, _D,
                                      C.c_int]
        lib.aio_integrate.restype = C.c_int
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def tableau() -> dict:
    c, b, bh, e = (np.zeros(7) for _ in range(4))
    a = np.zeros(49)
    load().aio_tableau(_ptr(c), _ptr(a), _ptr(b), _ptr(bh), _ptr(e))
    return {"c": c, "a": a.reshape(7, 7), "b": b, "bhat": bh, "e": e}


def force(sys_obj, t: float, y) -> np.ndarray:
    s = system(sys_obj)
    y = _f64(y)
    f = np.zeros(NSTATE)
    load().aio_force(C.byref(s), t, _ptr(y), _ptr(f))
    return f


def energy(sys_obj, t: float, y) -> float:
    s = system(sys_obj)
    return load().aio_energy(C.byref(s), t, _ptr(_f64(y)))


def spacing(t: float) -> float:
    return load().aio_spacing(t)


def initial_step(y0, f0, t0, tf, rtol, threshold, hmax) -> float:
    y0, f0 = _f64(y0), _f64(f0)
    return load().aio_initial_step(len(y0), _ptr(y0), _ptr(f0), t0, tf, rtol, threshold, hmax)


def error_norm(absh, eps, y, ynew, threshold) -> float:
    eps, y, ynew = _f64(eps), _f64(y), _f64(ynew)
    return load().aio_error_norm(len(y), absh, _ptr(eps), _ptr(y), _ptr(ynew), threshold)


def step_after_failure(absh, err, rtol, first_failure, hmin) -> float:
    return load().aio_step_after_failure(absh, err, rtol, int(first_failure), hmin)


def step_after_success(absh, err, rtol) -> float:
    return load().aio_step_after_success(absh, err, rtol)


def linear_attempt(Amat, t, h, y):
    Amat, y = _f64(Amat), _f64(y)
    ynew, eps = np.zeros_like(y), np.zeros_like(y)
    load().aio_linear_attempt(len(y), _ptr(Amat), t, h, _ptr(y), _ptr(ynew), _ptr(eps))
    return ynew, eps


def linear_ode45(Amat, t0, tf, y0, rtol, atol, hmax=0.0, max_steps=10**9, hist_cap=0):
    Amat, y0 = _f64(Amat), _f64(y0)
    yout = np.zeros_like(y0)
    run = Run()
    th, hh = np.zeros(max(hist_cap, 1)), np.zeros(max(hist_cap, 1))
    rc = load().aio_linear_ode45(len(y0), _ptr(Amat), t0, tf, _ptr(y0), rtol, atol, hmax,
                                 max_steps, _ptr(yout), C.byref(run), _ptr(th), _ptr(hh),
                                 hist_cap)
    out = run.as_dict()
    out["rc"] = rc
    n = min(run.nsteps, hist_cap)
    return yout, out, th[:n], hh[:n]


def rhs_attempt(fun, t, h, y):
    """One Dormand-Prince attempt of size h on y' = fun(t, y): (ynew, eps)."""
    y = _f64(y)
    ynew, eps = np.zeros_like(y), np.zeros_like(y)
    cb = _wrap_rhs(fun, len(y))
    load().aio_rhs_attempt(len(y), cb, None, t, h, _ptr(y), _ptr(ynew), _ptr(eps))
    return ynew, eps


def rhs_ode45(fun, t0, tf, y0, rtol, atol, hmax=0.0, max_steps=10**9, hist_cap=0):
    y0 = _f64(y0)
    yout = np.zeros_like(y0)
    run = Run()
    th, hh = np.zeros(max(hist_cap, 1)), np.zeros(max(hist_cap, 1))
    cb = _wrap_rhs(fun, len(y0))
    rc = load().aio_rhs_ode45(len(y0), cb, None, t0, tf, _ptr(y0), rtol, atol, hmax, max_steps,
                              _ptr(yout), C.byref(run), _ptr(th), _ptr(hh), hist_cap)
    out = run.as_dict()
    out["rc"] = rc
    n = min(run.nsteps, hist_cap)
    return yout, out, th[:n], hh[:n]


def integrate_one(sys_obj, t0, tf, y0, rtol, atol):
    s = system(sys_obj)
    y0 = _f64(y0)
    yf, ob = np.zeros(NSTATE), np.zeros(NOBS)
    rc = load().aio_integrate_one(C.byref(s), t0, tf, _ptr(y0), rtol, atol, _ptr(yf), _ptr(ob))
    return yf, ob, rc


def integrate(sys_obj, y0, t0, tmax, rtol, atol, nthreads: int = 0, n: int | None = None):
    """Integrate a (12, ld) ensemble (its first n columns; all by default).

    Returns (final (12, ld), obs (13, ld), rc); columns past n stay zero."""
    s = system(sys_obj)
    y0 = _f64(y0)
    if y0.ndim != 2 or y0.shape[0] != NSTATE:
        raise ValueError("y0 must have shape (12, ld)")
    ld = y0.shape[1]
    n = ld if n is None else n
    yf = np.zeros((NSTATE, ld))
    ob = np.zeros((NOBS, ld))
    rc = load().aio_integrate(C.byref(s), _ptr(y0), n, ld, t0, tmax, rtol, atol, _ptr(yf),
                              _ptr(ob), int(nthreads))
    return yf, ob, rc
