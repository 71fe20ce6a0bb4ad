"""FP64 CPU oracle for the minimum enclosing ball of balls (ripALM).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package; the product library never
does, and the two share no code.  The arithmetic lives in ``meb_oracle.c``
(plain C, double precision, long-double sums in ball order); this module
only marshals numpy arrays into it.  ``brute.py`` holds the exhaustive
small-instance solver used to pin the oracle.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int64)


class Params(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("sigma0", ctypes.c_double), ("sigma_growth", ctypes.c_double),
                ("sigma_max", ctypes.c_double), ("tau", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("max_inner", ctypes.c_int), ("max_ls", ctypes.c_int),
                ("stall_outer", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int), ("inner", ctypes.c_int), ("ls_evals", ctypes.c_int),
                ("kkt", ctypes.c_double), ("L", ctypes.c_double), ("rbar", ctypes.c_double),
                ("r_fixed", ctypes.c_double), ("kkt_parts", ctypes.c_double * 5)]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        L.orc_soc_project.restype = ctypes.c_int
        L.orc_soc_project.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.orc_soc_jacobian.restype = ctypes.c_int
        L.orc_soc_jacobian.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.orc_soc_dist.restype = ctypes.c_double
        L.orc_soc_dist.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
        L.orc_al_eval.restype = ctypes.c_int
        L.orc_al_eval.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_double,
                                  ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _ip, _dp]
        L.orc_kkt_max.restype = ctypes.c_double
        L.orc_kkt_max.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_screen.restype = ctypes.c_int64
        L.orc_screen.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, ctypes.c_double, _dp, ctypes.c_double,
                                 _ip, _dp]
        L.orc_check_feasible.restype = ctypes.c_double
        L.orc_check_feasible.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, ctypes.c_double, _dp,
                                         ctypes.c_double, _ip, _ip, ctypes.c_int64, _ip]
        L.orc_chol_solve.restype = ctypes.c_int
        L.orc_chol_solve.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.orc_default_params.restype = None
        L.orc_default_params.argtypes = [ctypes.POINTER(Params)]
        L.orc_ripalm.restype = ctypes.c_int
        L.orc_ripalm.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, ctypes.POINTER(Params), _dp, _dp, _dp,
                                 _dp, _dp, _dp, ctypes.POINTER(Stats)]
        _lib = L
    return _lib


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _pi(a):
    return None if a is None else a.ctypes.data_as(_ip)


def soc_project(t, s):
    """Projection of (t, s) onto the second-order cone; returns (pt, ps, case)."""
    s = _f64(np.atleast_1d(s))
    ps = np.empty_like(s)
    pt = ctypes.c_double()
    case = lib().orc_soc_project(len(s), float(t), _p(s), ctypes.byref(pt), _p(ps))
    return pt.value, ps, case


def soc_jacobian(t, s):
    s = _f64(np.atleast_1d(s))
    P = np.empty((len(s) + 1, len(s) + 1))
    case = lib().orc_soc_jacobian(len(s), float(t), _p(s), _p(P))
    return P, case


def soc_dist(t, s):
    s = _f64(np.atleast_1d(s))
    return lib().orc_soc_dist(len(s), float(t), _p(s))


def al_eval(C, R, U, V, x, xbar, sigma, tau, want_h=True, want_mult=True):
    """Direct per-ball evaluation of Psi, grad Psi, H, the multiplier update
    and sum ||(u+ - u, v+ - v)||^2.  Returns a dict."""
    C = _f64(C)
    m, d = C.shape
    R, U, V = _f64(R), _f64(U), _f64(V)
    x, xbar = _f64(x), _f64(xbar)
    psi = ctypes.c_double()
    dm = ctypes.c_double()
    rs = ctypes.c_double()
    g = np.empty(d + 1)
    H = np.empty((d + 1, d + 1)) if want_h else None
    Un = np.empty(m) if want_mult else None
    Vn = np.empty((m, d)) if want_mult else None
    cnt = np.zeros(3, dtype=np.int64)
    lib().orc_al_eval(m, d, _p(C), _p(R), _p(U), _p(V), _p(x), _p(xbar), float(sigma), float(tau),
                      ctypes.byref(psi), _p(g), _p(H), _p(Un), _p(Vn), ctypes.byref(dm), _pi(cnt), ctypes.byref(rs))
    return dict(psi=psi.value, g=g, H=H, U=Un, V=Vn, dmult=dm.value, counts=cnt, rscale=rs.value)


def kkt_max(C, R, U, V, x):
    C = _f64(C)
    m, d = C.shape
    parts = np.empty(5)
    v = lib().orc_kkt_max(m, d, _p(C), _p(_f64(R)), _p(_f64(U)), _p(_f64(V)), _p(_f64(x)), _p(parts))
    return v, parts


def screen(C, R, rhat, chat, tol_red):
    C = _f64(C)
    m, d = C.shape
    keep = np.empty(m, dtype=np.int64)
    slack = np.empty(m)
    n = lib().orc_screen(m, d, _p(C), _p(_f64(R)), float(rhat), _p(_f64(chat)), float(tol_red), _pi(keep),
                         _p(slack))
    return keep[:n].copy(), slack


def check_feasible(C, R, r, c, eps):
    C = _f64(C)
    m, d = C.shape
    viol = np.empty(m, dtype=np.int64)
    am = ctypes.c_int64()
    nv = ctypes.c_int64()
    dmax = lib().orc_check_feasible(m, d, _p(C), _p(_f64(R)), float(r), _p(_f64(c)), float(eps),
                                    ctypes.byref(am), _pi(viol), m, ctypes.byref(nv))
    return dmax, am.value, viol[:nv.value].copy()


def chol_solve(A, b):
    A = _f64(A)
    b = _f64(b)
    x = np.empty_like(b)
    rc = lib().orc_chol_solve(len(b), _p(A), _p(b), _p(x))
    if rc != 0:
        raise np.linalg.LinAlgError("matrix is not positive definite")
    return x


def default_params(**kw):
    p = Params()
    lib().orc_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def ripalm(C, R=None, params=None, x0=None, U0=None, V0=None, want_mult=False, **kw):
    """Runs the oracle's ripALM.  Returns (r, c, stats dict[, U, V])."""
    C = _f64(C)
    m, d = C.shape
    p = params if params is not None else default_params(**kw)
    x = np.empty(d + 1)
    U = np.empty(m) if want_mult else None
    V = np.empty((m, d)) if want_mult else None
    st = Stats()
    rc = lib().orc_ripalm(m, d, _p(C), _p(_f64(R)), ctypes.byref(p), _p(_f64(x0)), _p(_f64(U0)), _p(_f64(V0)),
                          _p(x), _p(U), _p(V), ctypes.byref(st))
    stats = dict(status=rc, outer=st.outer, inner=st.inner, ls_evals=st.ls_evals, kkt=st.kkt, L=st.L,
                 rbar=st.rbar, r_fixed=st.r_fixed, kkt_parts=list(st.kkt_parts))
    if want_mult:
        return x[0], x[1:].copy(), stats, U, V
    return x[0], x[1:].copy(), stats


def prepare_f32(C, R, origin):
    """The precision preparation written out: each row minus the origin in
    FP64, rounded to nearest FP32; radii rounded to FP32; and the scale
    L = max_i ||c_i - origin|| + r_i."""
    C = _f64(C)
    E = C - np.asarray(origin, dtype=np.float64)[None, :]
    C32 = E.astype(np.float32)
    R32 = None if R is None else _f64(R).astype(np.float32)
    L, _, _ = check_feasible(C, R, 0.0, origin, np.inf)
    return C32, R32, L
