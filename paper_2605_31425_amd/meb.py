"""ctypes binding of libmeb.so (include/meb.h).

Argument marshalling only: every step of the solver runs in the HIP library.
torch supplies device memory (tensors are passed by ``data_ptr()``) and the
current stream.  Importing this module on a machine without the built
library raises immediately; there is no fallback path.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmeb.so")

MEB_OK = 0
MEB_WARN_MAXITER = 1
MEB_ERR_ARG, MEB_ERR_HIP, MEB_ERR_WORKSPACE, MEB_ERR_NUMERIC, MEB_ERR_UNSUPPORTED = -1, -2, -3, -4, -5
MEB_F64 = 0
MEB_F32 = 1
MEB_MODE_FP64 = 0
MEB_MODE_MIXED = 1
MEB_HESS_AUTO, MEB_HESS_F64, MEB_HESS_MFMA_F64, MEB_HESS_MFMA_F32, MEB_HESS_MFMA_BF16 = 0, 1, 2, 3, 4
_HESS = {"auto": 0, "f64": 1, "mfma_f64": 2, "mfma_f32": 3, "mfma_bf16": 4}
WANT_PSI, WANT_GRAD, WANT_HESS, WANT_MULT, WANT_DMULT, WANT_KKT = 1, 2, 4, 8, 16, 32
WANT_ALL = 63

EXPORTS = ["meb_default_options", "meb_last_error", "meb_source_hash", "meb_workspace_size", "meb_eval_workspace_size", "meb_solve",
           "meb_al_eval", "meb_hess_vec", "meb_screen", "meb_check_feasible", "meb_check_feasible_noalloc",
           "meb_prepare_f32",
           "meb_chol_workspace_size",
           "meb_chol_solve", "meb_server_create", "meb_server_submit", "meb_server_poll", "meb_server_info",
           "meb_server_destroy", "meb_sched_simulate"]


class Options(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("sigma0", ctypes.c_double), ("sigma_growth", ctypes.c_double),
                ("sigma_max", ctypes.c_double), ("tau", ctypes.c_double), ("tol_kkt", ctypes.c_double),
                ("tol_kkt_low", ctypes.c_double), ("tol_red", ctypes.c_double), ("eps_feas_rel", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("max_inner", ctypes.c_int32), ("max_ls", ctypes.c_int32),
                ("max_reinsert", ctypes.c_int32), ("mode", ctypes.c_int32), ("stall_outer", ctypes.c_int32),
                ("verbose", ctypes.c_int32), ("profile", ctypes.c_int32), ("hess", ctypes.c_int32),
                ("first_order_outer", ctypes.c_int32), ("newton", ctypes.c_int32),
                ("cg_max_iter", ctypes.c_int32), ("cg_tol", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int32 * 2), ("inner", ctypes.c_int32 * 2), ("passes", ctypes.c_int32 * 2),
                ("kkt", ctypes.c_double * 2), ("L", ctypes.c_double), ("rbar", ctypes.c_double),
                ("delta_max", ctypes.c_double), ("n_red", ctypes.c_int64), ("reinsert_rounds", ctypes.c_int32),
                ("status", ctypes.c_int32), ("ms_total", ctypes.c_double), ("ms_phase", ctypes.c_double * 4),
                ("pass_ms", ctypes.c_double * 2), ("pass_bytes", ctypes.c_double * 2),
                ("pass_launches", ctypes.c_int32 * 2), ("reserved", ctypes.c_int32),
                ("mid_rows", ctypes.c_double * 2), ("mid_rows_max", ctypes.c_double * 2),
                ("newton_shifted", ctypes.c_int32 * 2), ("inner_breaks", ctypes.c_int32 * 2),
                ("first_order_steps", ctypes.c_int32 * 2), ("cg_iterations", ctypes.c_int32 * 2)]

    def as_dict(self):
        return dict(outer=list(self.outer), inner=list(self.inner), passes=list(self.passes), kkt=list(self.kkt),
                    L=self.L, rbar=self.rbar, delta_max=self.delta_max, n_red=self.n_red,
                    reinsert_rounds=self.reinsert_rounds, status=self.status, ms_total=self.ms_total,
                    ms_phase=list(self.ms_phase), pass_ms=list(self.pass_ms), pass_bytes=list(self.pass_bytes),
                    pass_launches=list(self.pass_launches), mid_rows=list(self.mid_rows),
                    mid_rows_max=list(self.mid_rows_max), newton_shifted=list(self.newton_shifted),
                    inner_breaks=list(self.inner_breaks), first_order_steps=list(self.first_order_steps),
                    cg_iterations=list(self.cg_iterations))


class ServerResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("tag", ctypes.c_int64), ("m", ctypes.c_int64), ("d", ctypes.c_int32),
                ("status", ctypes.c_int32), ("r", ctypes.c_double), ("t_submit_ms", ctypes.c_double),
                ("t_admit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double), ("stats", Stats),
                ("message", ctypes.c_char * 128)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int32), ("active", ctypes.c_int32), ("pool_used", ctypes.c_uint64),
                ("pool_peak", ctypes.c_uint64), ("pool_capacity", ctypes.c_uint64), ("ticks", ctypes.c_int64),
                ("mean_tick_items", ctypes.c_double), ("message", ctypes.c_char * 128)]


class MebError(RuntimeError):
    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_szp = ctypes.POINTER(ctypes.c_size_t)


def _load():
    if not os.path.exists(LIB_PATH):
        raise MebError(f"{LIB_PATH} is not built; run paper_2605_31425_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    L.meb_default_options.argtypes = [ctypes.POINTER(Options)]
    L.meb_last_error.restype = ctypes.c_char_p
    L.meb_source_hash.restype = ctypes.c_char_p
    L.meb_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Options), _szp]
    L.meb_eval_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _szp]
    L.meb_solve.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Options), _vp,
                            ctypes.c_size_t, _dp, _dp, _vp, _vp, ctypes.POINTER(Stats), _vp]
    L.meb_al_eval.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _dp, _dp,
                              ctypes.c_double, ctypes.c_double, _dp, ctypes.c_int32, _dp, ctypes.c_uint32, _dp, _dp,
                              _dp, _dp, _vp, _vp, _dp, _dp, _vp, ctypes.c_size_t, _vp]
    L.meb_screen.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _dp,
                             ctypes.c_double, _vp, _i64p, _vp, _vp, ctypes.c_size_t, _vp]
    L.meb_check_feasible.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _dp,
                                     ctypes.c_double, _dp, _i64p, _vp, ctypes.c_int64, _i64p, _vp, ctypes.c_size_t,
                                     _vp]
    L.meb_hess_vec.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _dp,
                               ctypes.c_double, ctypes.c_double, _dp, _dp, _vp, ctypes.c_size_t, _vp]
    L.meb_check_feasible_noalloc.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_double, _dp, ctypes.c_double, _dp, _i64p, _vp, ctypes.c_int64,
                                             _i64p, _vp]
    L.meb_prepare_f32.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _dp, _vp, _vp, _dp, _vp, ctypes.c_size_t,
                                  _vp]
    L.meb_chol_workspace_size.argtypes = [ctypes.c_int32, _szp]
    L.meb_chol_solve.argtypes = [ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.meb_server_create.argtypes = [_vp, ctypes.c_size_t, ctypes.POINTER(Options), ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(_vp)]
    L.meb_server_submit.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                    _dp, _i64p]
    L.meb_server_poll.argtypes = [_vp, ctypes.POINTER(ServerResult), ctypes.c_int32, ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_int32)]
    L.meb_server_info.argtypes = [_vp, ctypes.POINTER(ServerStats)]
    L.meb_server_destroy.argtypes = [_vp]
    _u64p = ctypes.POINTER(ctypes.c_uint64)
    L.meb_sched_simulate.argtypes = [ctypes.c_int32, _dp, _dp, _u64p, ctypes.c_uint64, ctypes.c_int32, _dp, _dp,
                                     _u64p]
    return L


lib = _load()


def source_hash():
    """The source hash compiled into the loaded libmeb.so."""
    return lib.meb_source_hash().decode()


def _check(rc):
    if rc < 0:
        raise MebError(f"libmeb error {rc}: {lib.meb_last_error().decode()}", rc)
    return rc


def options(**kw):
    o = Options()
    lib.meb_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "mode" and isinstance(v, str):
            v = {"fp64": MEB_MODE_FP64, "mixed": MEB_MODE_MIXED}[v]
        if k == "hess" and isinstance(v, str):
            v = _HESS[v]
        if k == "newton" and isinstance(v, str):
            v = {"dense": 0, "cg": 1}[v]
        setattr(o, k, v)
    return o


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    if t.dtype == torch.float64:
        return MEB_F64
    if t.dtype == torch.float32:
        return MEB_F32
    raise MebError("centers must be float64 or float32")


def _host(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _workspace(nbytes, device):
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def solve(C, R=None, opts=None, want_mult=False, workspace=None, **kw):
    """meb_solve on device tensors C (m x d float64) and R (m or None).
    Returns (r, c numpy, stats dict[, U, V tensors])."""
    assert C.is_cuda and C.is_contiguous() and C.dim() == 2
    m, d = C.shape
    o = opts if opts is not None else options(**kw)
    nb = ctypes.c_size_t()
    _check(lib.meb_workspace_size(m, d, _dtype_code(C), ctypes.byref(o), ctypes.byref(nb)))
    ws = workspace if workspace is not None and workspace.numel() >= nb.value else _workspace(nb.value, C.device)
    r = ctypes.c_double()
    c = np.empty(d)
    U = torch.empty(m, dtype=torch.float64, device=C.device) if want_mult else None
    V = torch.empty((m, d), dtype=torch.float64, device=C.device) if want_mult else None
    st = Stats()
    rc = _check(lib.meb_solve(_ptr(C), _ptr(R), m, d, _dtype_code(C), ctypes.byref(o), _ptr(ws), ws.numel(),
                              ctypes.byref(r), c.ctypes.data_as(_dp), _ptr(U), _ptr(V), ctypes.byref(st), _stream()))
    out = (r.value, c, dict(st.as_dict(), rc=rc))
    return out + (U, V) if want_mult else out


def al_eval(C, R, U, V, x, xbar, sigma, tau, direction=None, etas=(), want=WANT_ALL):
    """meb_al_eval.  Returns a dict with psi, psi_trial, g, H, U_new, V_new, dmult, kkt."""
    m, d = C.shape
    dt = _dtype_code(C)
    nb = ctypes.c_size_t()
    _check(lib.meb_eval_workspace_size(m, d, dt, ctypes.byref(nb)))
    ws = _workspace(nb.value, C.device)
    xh, xp = _host(x)
    xbh, xbp = _host(xbar)
    dh, dp = _host(direction) if direction is not None else (None, None)
    eh, ep = _host(etas) if len(etas) else (None, None)
    psi = ctypes.c_double()
    dm = ctypes.c_double()
    pt = np.empty(max(len(etas), 1))
    g = np.empty(d + 1)
    H = np.empty((d + 1, d + 1))
    kkt = np.empty(5)
    Un = torch.empty(m, dtype=C.dtype, device=C.device) if want & WANT_MULT else None
    Vn = torch.empty((m, d), dtype=C.dtype, device=C.device) if want & WANT_MULT else None
    _check(lib.meb_al_eval(_ptr(C), _ptr(R), _ptr(U), _ptr(V), m, d, dt, xp, xbp, float(sigma), float(tau), dp,
                           len(etas), ep, want, ctypes.byref(psi), pt.ctypes.data_as(_dp) if len(etas) else None,
                           g.ctypes.data_as(_dp), H.ctypes.data_as(_dp), _ptr(Un), _ptr(Vn), ctypes.byref(dm),
                           kkt.ctypes.data_as(_dp), _ptr(ws), ws.numel(), _stream()))
    return dict(psi=psi.value, psi_trial=pt[:len(etas)], g=g, H=H, U=Un, V=Vn, dmult=dm.value, kkt=kkt)


def screen(C, R, r_hat, c_hat, tol_red, want_slack=False):
    m, d = C.shape
    dt = _dtype_code(C)
    nb = ctypes.c_size_t()
    _check(lib.meb_eval_workspace_size(m, d, dt, ctypes.byref(nb)))
    ws = _workspace(nb.value, C.device)
    keep = torch.empty(m, dtype=torch.int64, device=C.device)
    slack = torch.empty(m, dtype=torch.float64, device=C.device) if want_slack else None
    n = ctypes.c_int64()
    ch, cp = _host(c_hat)
    _check(lib.meb_screen(_ptr(C), _ptr(R), m, d, dt, float(r_hat), cp, float(tol_red), _ptr(keep), ctypes.byref(n),
                          _ptr(slack), _ptr(ws), ws.numel(), _stream()))
    return keep[:n.value], slack


def check_feasible(C, R, r, c, eps, viol_cap=None):
    m, d = C.shape
    dt = _dtype_code(C)
    nb = ctypes.c_size_t()
    _check(lib.meb_eval_workspace_size(m, d, dt, ctypes.byref(nb)))
    ws = _workspace(nb.value, C.device)
    cap = m if viol_cap is None else viol_cap
    viol = torch.empty(max(cap, 1), dtype=torch.int64, device=C.device)
    dmax = ctypes.c_double()
    am = ctypes.c_int64()
    nv = ctypes.c_int64()
    ch, cp = _host(c)
    _check(lib.meb_check_feasible(_ptr(C), _ptr(R), m, d, dt, float(r), cp, float(eps), ctypes.byref(dmax),
                                  ctypes.byref(am), _ptr(viol) if cap > 0 else None, cap, ctypes.byref(nv), _ptr(ws),
                                  ws.numel(), _stream()))
    return dmax.value, am.value, viol[:min(nv.value, cap)], nv.value


def hess_vec(C, R, U, V, x, sigma, tau, q):
    """meb_hess_vec: the generalized Hessian at x times q, without forming H."""
    m, d = C.shape
    dt = _dtype_code(C)
    nb = ctypes.c_size_t()
    _check(lib.meb_eval_workspace_size(m, d, dt, ctypes.byref(nb)))
    ws = _workspace(nb.value, C.device)
    xh, xp = _host(x)
    qh, qp = _host(q)
    out = np.empty(d + 1)
    _check(lib.meb_hess_vec(_ptr(C), _ptr(R), _ptr(U), _ptr(V), m, d, dt, xp, float(sigma), float(tau), qp,
                            out.ctypes.data_as(_dp), _ptr(ws), ws.numel(), _stream()))
    return out


def check_feasible_noalloc(C, R, r, c, eps, viol_idx=None):
    """meb_check_feasible_noalloc: like check_feasible, with the library's
    fixed scratch instead of a workspace.  viol_idx (device int64 tensor,
    nullable) receives the first viol_idx.numel() violated indices."""
    m, d = C.shape
    dt = _dtype_code(C)
    cap = 0 if viol_idx is None else viol_idx.numel()
    dmax = ctypes.c_double()
    am = ctypes.c_int64()
    nv = ctypes.c_int64()
    ch, cp = _host(c)
    _check(lib.meb_check_feasible_noalloc(_ptr(C), _ptr(R), m, d, dt, float(r), cp, float(eps), ctypes.byref(dmax),
                                          ctypes.byref(am), _ptr(viol_idx) if cap > 0 else None, cap,
                                          ctypes.byref(nv), _stream()))
    return dmax.value, am.value, nv.value


def prepare_f32(C, R, origin=None):
    m, d = C.shape
    nb = ctypes.c_size_t()
    _check(lib.meb_eval_workspace_size(m, d, MEB_F64, ctypes.byref(nb)))
    ws = _workspace(nb.value, C.device)
    C32 = torch.empty((m, d), dtype=torch.float32, device=C.device)
    R32 = torch.empty(m, dtype=torch.float32, device=C.device) if R is not None else None
    L = ctypes.c_double()
    op = _host(origin)[1] if origin is not None else None
    _check(lib.meb_prepare_f32(_ptr(C), _ptr(R), m, d, op, _ptr(C32), _ptr(R32), ctypes.byref(L), _ptr(ws),
                               ws.numel(), _stream()))
    return C32, R32, L.value


def chol_solve(H, b):
    n = b.shape[0]
    nb = ctypes.c_size_t()
    _check(lib.meb_chol_workspace_size(n, ctypes.byref(nb)))
    ws = _workspace(nb.value, H.device)
    y = torch.empty_like(b)
    _check(lib.meb_chol_solve(n, _ptr(H), _ptr(b), _ptr(y), _ptr(ws), ws.numel(), _stream()))
    return y


class Server:
    """meb_server_* on a device pool of `pool_bytes`.  submit() keeps the
    request's tensors and its host center buffer alive until its result is
    polled."""

    def __init__(self, pool_bytes, opts=None, max_active=128, max_d=256, device="cuda", **kw):
        o = opts if opts is not None else options(**kw)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        if self.pool.data_ptr() % 256:
            raise MebError("pool allocation is not 256-byte aligned")
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(lib.meb_server_create(_ptr(self.pool), self.pool.numel(), ctypes.byref(o), max_active, max_d,
                                     ctypes.byref(h)))
        self.h = h
        self.live = {}

    def submit(self, C, R=None, tag=0):
        assert C.is_cuda and C.is_contiguous() and C.dim() == 2
        m, d = C.shape
        c_out = np.zeros(d)
        t = ctypes.c_int64()
        _check(lib.meb_server_submit(self.h, _ptr(C), _ptr(R), m, d, _dtype_code(C), int(tag),
                                     c_out.ctypes.data_as(_dp), ctypes.byref(t)))
        self.live[t.value] = (C, R, c_out)
        return t.value

    def poll(self, wait_ms=0, cap=256):
        buf = (ServerResult * cap)()
        n = ctypes.c_int32()
        _check(lib.meb_server_poll(self.h, buf, cap, int(wait_ms), ctypes.byref(n)))
        out = []
        for k in range(n.value):
            r = buf[k]
            _, _, c = self.live.pop(r.ticket, (None, None, None))
            out.append(dict(ticket=r.ticket, tag=r.tag, m=r.m, d=r.d, status=r.status, r=r.r, c=c,
                            t_submit_ms=r.t_submit_ms, t_admit_ms=r.t_admit_ms, t_done_ms=r.t_done_ms,
                            stats=r.stats.as_dict(), message=r.message.decode()))
        return out

    def info(self):
        st = ServerStats()
        _check(lib.meb_server_info(self.h, ctypes.byref(st)))
        return {k: (getattr(st, k).decode() if k == "message" else getattr(st, k)) for k, _ in st._fields_}

    def close(self):
        if self.h:
            _check(lib.meb_server_destroy(self.h))
            self.h = None
            self.live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sched_simulate(arrival, service, nbytes, pool_bytes, max_active):
    """meb_sched_simulate: the server's admission policy on a simulated clock.
    Returns (t_admit, t_done, offset) arrays."""
    arrival = np.ascontiguousarray(arrival, dtype=np.float64)
    service = np.ascontiguousarray(service, dtype=np.float64)
    nbytes = np.ascontiguousarray(nbytes, dtype=np.uint64)
    n = arrival.shape[0]
    ta, td = np.empty(n), np.empty(n)
    off = np.empty(n, dtype=np.uint64)
    u64 = ctypes.POINTER(ctypes.c_uint64)
    _check(lib.meb_sched_simulate(n, arrival.ctypes.data_as(_dp), service.ctypes.data_as(_dp),
                                  nbytes.ctypes.data_as(u64), int(pool_bytes), int(max_active),
                                  ta.ctypes.data_as(_dp), td.ctypes.data_as(_dp), off.ctypes.data_as(u64)))
    return ta, td, off
