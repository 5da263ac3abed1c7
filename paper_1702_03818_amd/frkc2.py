"""Python binding of libfrkc2 (the C ABI in include/frkc2.h).

Argument marshalling only: every step of the superstep runs in the library's
HIP kernels. Tensors are torch float64 CUDA (HIP) tensors, contiguous; the
binding passes their device pointers, the current torch stream, and a device
workspace it allocates through torch (cached per device and size).

The functions keep the C names. Grids are anything with the attributes
ndim, n (nx, ny, nz), h, bc, op and d_const (a workloads.Problem works) or a
dict with those keys.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrkc2.so")

FRKC2_OK = 0
FRKC2_WQBOUND = 1
STATUS_NAMES = {0: "OK", 1: "WQBOUND", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP",
                -4: "EUNSTABLE", -5: "ENONFINITE", -6: "ETIMEOUT",
                -7: "EDISABLED"}
WS_STEP = 0
NOALLOC_MAX_VALUES = 2097152   # largest state frkc2_step_noalloc accepts (2^21 values)
WS_ADJOINT = 1
WS_ADAPT = 2
WS_STAGES = 3
WS_ADJOINT_STORED = 4
RED_SUMSQ, RED_SUM, RED_MAXSQ, RED_SUMSQDIFF, RED_DOT = 0, 1, 2, 3, 4
OPT_TBLOCK = 1
OPT_TILE = 3
OPT_CLEAR_TUNED = 4
OPT_ZCHUNK = 5
OPT_BATCH_K3 = 6
OPT_ADJ_STAGES = 9
OPT_BATCH_COLS = 7
OPT_BATCH_K2 = 8


class Frkc2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("bc", ctypes.c_int), ("op", ctypes.c_int), ("d_const", ctypes.c_double),
                ("vel", ctypes.c_double * 3)]


class CoeffInfo(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("beta_bar", ctypes.c_double),
                ("q_realised", ctypes.c_double), ("mu_re", ctypes.c_double),
                ("mu_im", ctypes.c_double), ("n_shrink", ctypes.c_int),
                ("q_bound_met", ctypes.c_int)]


class StepStats(ctypes.Structure):
    _fields_ = [("T_last", ctypes.c_double), ("rho_last", ctypes.c_double),
                ("im_ratio", ctypes.c_double), ("supersteps", ctypes.c_int)]


class AdaptStats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("T_next", ctypes.c_double),
                ("err_last", ctypes.c_double), ("stages", ctypes.c_longlong),
                ("attempts", ctypes.c_int), ("accepted", ctypes.c_int),
                ("rejected", ctypes.c_int), ("s_last", ctypes.c_int)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tblock", ctypes.c_int), ("tile", ctypes.c_int), ("zchunk", ctypes.c_int),
                ("candidates", ctypes.c_int), ("ms_best", ctypes.c_double),
                ("ms_default", ctypes.c_double)]


class BatchTuneResult(ctypes.Structure):
    _fields_ = [("k3", ctypes.c_int), ("cols3", ctypes.c_int), ("k2", ctypes.c_int),
                ("candidates", ctypes.c_int), ("ms_best", ctypes.c_double),
                ("ms_default", ctypes.c_double)]


_lib = None
_VP = ctypes.c_void_p
USER_F = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_longlong,
                          ctypes.c_void_p, ctypes.c_void_p)
_DP = ctypes.POINTER(ctypes.c_double)
USER_RHO = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p,
                            ctypes.c_void_p, _DP)

_SIGS = {
    "frkc2_coeffs": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, _DP, _DP, ctypes.POINTER(CoeffInfo)]),
    "frkc4_coeffs": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, _DP, _DP, ctypes.POINTER(CoeffInfo)]),
    "frkc4s_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid)]),
    "frkc4s_step": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_int, _VP,
                                   ctypes.c_size_t, _VP]),
    "frkc2_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), ctypes.c_int, ctypes.c_int]),
    "frkc2_rho_bound": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, _VP, _DP, _VP, ctypes.c_size_t, _VP]),
    "frkc2_step": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, _VP, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_double, ctypes.c_int, _VP, ctypes.c_size_t,
                                  _VP, ctypes.POINTER(StepStats)]),
    "frkc2_step_noalloc": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, _VP, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_int, _VP, ctypes.POINTER(StepStats)]),
    "frkc2_step_adjoint": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, _VP, ctypes.c_double,
                                          ctypes.c_int, ctypes.c_double, _VP, _VP, _VP, _VP,
                                          ctypes.c_size_t, _VP]),
    "frkc2_step_store": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, _VP, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_double, _VP, ctypes.c_size_t, _VP,
                                        ctypes.c_size_t, _VP]),
    "frkc2_step_adjoint_stored": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, ctypes.c_size_t, _VP,
                                                 ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                                 _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "frkc2_batched_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.POINTER(Grid),
                                                        ctypes.POINTER(ctypes.c_int)]),
    "frkc2_step_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Grid),
                                          ctypes.POINTER(_VP), ctypes.POINTER(_VP), _DP,
                                          ctypes.POINTER(ctypes.c_int), ctypes.c_double, _VP,
                                          ctypes.c_size_t, _VP]),
    "frkc2_batched_autotune": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Grid),
                                              ctypes.POINTER(_VP), ctypes.POINTER(_VP), _DP,
                                              ctypes.POINTER(ctypes.c_int), ctypes.c_double,
                                              ctypes.c_int, _VP, ctypes.c_size_t, _VP,
                                              ctypes.POINTER(BatchTuneResult)]),
    "frkc2_batched_config": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Grid),
                                            ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_int)]),
    "frkc2_batched_status": (ctypes.c_int, [_VP, _VP]),
    "frkc2_batched_release": (ctypes.c_int, [_VP]),
    "frkc2_reduce": (ctypes.c_int, [ctypes.c_int, _VP, _VP, ctypes.c_size_t, _DP, _VP,
                                    ctypes.c_size_t, _VP]),
    "frkc2_integrate": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, _VP, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, _VP, ctypes.c_size_t, _VP, _DP, ctypes.c_int,
                                       ctypes.POINTER(AdaptStats)]),
    "frkc2_step_user": (ctypes.c_int, [ctypes.c_longlong, _VP, USER_F, _VP, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       _VP, ctypes.c_size_t, _VP]),
    "frkc2_user_workspace_bytes": (ctypes.c_size_t, [ctypes.c_longlong, ctypes.c_int]),
    "frkc2_integrate_user": (ctypes.c_int, [ctypes.c_longlong, _VP, USER_F, USER_RHO,
                                            ctypes.c_double, _VP, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int, _VP,
                                            ctypes.c_size_t, _VP, _DP, ctypes.c_int,
                                            ctypes.POINTER(AdaptStats)]),
    "frkc2_autotune": (ctypes.c_int, [ctypes.POINTER(Grid), _VP, _VP, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int, _VP, ctypes.c_size_t, _VP,
                                      ctypes.POINTER(TuneResult)]),
    "frkc2_write_table": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_double, ctypes.c_int]),
    "frkc2_set_option": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "frkc2_stream_copy": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, _VP]),
    "frkc2_last_error": (ctypes.c_char_p, []),
    "frkc2_version": (ctypes.c_char_p, []),
}


def load():
    """Load libfrkc2.so (built in-tree). Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfrkc2.so is not built: run `python -m paper_1702_03818_amd.build` "
                               "(or __graft_entry__.build()) first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc < 0:
        raise Frkc2Error(rc, load().frkc2_last_error().decode())
    return rc


def make_grid(g) -> Grid:
    if isinstance(g, Grid):
        return g
    get = (lambda k: g[k]) if isinstance(g, dict) else (lambda k: getattr(g, k))
    n = list(get("n")) + [1] * (3 - len(get("n")))
    try:
        vel = list(get("vel"))
    except (KeyError, AttributeError):
        vel = []
    vel = [float(v) for v in vel] + [0.0] * (3 - len(vel))
    return Grid(int(get("ndim")), (ctypes.c_int * 3)(*[int(v) for v in n[:3]]), float(get("h")),
                int(get("bc")), int(get("op")), float(get("d_const")),
                (ctypes.c_double * 3)(*vel[:3]))


# ---- device plumbing (torch) ----

_ws_cache = {}


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def _forget(k):
    """Drop a cached workspace; the library's batched graph keyed on its address goes first
    (torch may hand the same address to the next buffer)."""
    buf = _ws_cache.pop(k, None)
    if buf is not None and k[1] == "batched" and _lib is not None:
        _lib.frkc2_batched_release(ctypes.c_void_p(buf.data_ptr()))


def workspace(nbytes: int, device=None, key="default"):
    """A cached uint8 device buffer of at least nbytes (grown on demand)."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    k = (dev.index, key)
    buf = _ws_cache.get(k)
    if buf is None or buf.numel() < nbytes:
        _forget(k)
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)
        _ws_cache[k] = buf
    return buf


def release_workspaces():
    for k in list(_ws_cache):
        _forget(k)


# ---- the ABI ----

def frkc2_coeffs(s: int, nu: float = 0.01):
    """Returns (a_re, a_im, info dict, status). Host only."""
    lib = load()
    re = np.zeros(s)
    im = np.zeros(s)
    info = CoeffInfo()
    rc = _check(lib.frkc2_coeffs(int(s), float(nu), re.ctypes.data_as(_DP), im.ctypes.data_as(_DP),
                                 ctypes.byref(info)))
    d = {f: getattr(info, f) for f, _ in CoeffInfo._fields_}
    return re, im, d, rc


def frkc4_coeffs(s: int, nu: float = 0.01):
    """Fourth-order stepsizes: returns (a_re, a_im, info dict, status). Host only."""
    lib = load()
    re = np.zeros(s)
    im = np.zeros(s)
    info = CoeffInfo()
    rc = _check(lib.frkc4_coeffs(int(s), float(nu), re.ctypes.data_as(_DP), im.ctypes.data_as(_DP),
                                 ctypes.byref(info)))
    d = {f: getattr(info, f) for f, _ in CoeffInfo._fields_}
    return re, im, d, rc


def frkc4s_step(grid, w, T, s, nsub=4, nu=0.01, nsteps=1, stream=None, ws=None):
    """nsteps steps of the split fourth-order scheme on the Brusselator state w (in place)."""
    lib = load()
    g = make_grid(grid)
    need = lib.frkc4s_workspace_bytes(ctypes.byref(g))
    if need == 0:
        _check(-1)
    buf = ws if ws is not None else workspace(need, key="split")
    return _check(lib.frkc4s_step(ctypes.byref(g), _ptr(w), float(T), int(s), int(nsub), float(nu),
                                  int(nsteps), ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                  _stream_ptr(stream)))


def frkc2_workspace_bytes(grid, s: int, flags: int = WS_STEP) -> int:
    g = make_grid(grid)
    return int(load().frkc2_workspace_bytes(ctypes.byref(g), int(s), int(flags)))


def frkc2_rho_bound(grid, w=None, D=None, stream=None) -> float:
    lib = load()
    g = make_grid(grid)
    ws = workspace(64 * 1024)
    rho = ctypes.c_double()
    _check(lib.frkc2_rho_bound(ctypes.byref(g), _ptr(w), _ptr(D), ctypes.byref(rho),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    return rho.value


def frkc2_step(grid, w, D=None, T=0.0, cfl=0.0, s=16, nu=0.01, nsteps=1, stream=None,
               stats=False, ws=None):
    """nsteps supersteps in place on w. Returns the stats dict if stats=True, else the status."""
    lib = load()
    g = make_grid(grid)
    need = lib.frkc2_workspace_bytes(ctypes.byref(g), int(s), WS_STEP)
    if need == 0:
        _check(-1)
    buf = ws if ws is not None else workspace(need)
    st = StepStats() if stats else None
    rc = _check(lib.frkc2_step(ctypes.byref(g), _ptr(w), _ptr(D), float(T), float(cfl), int(s),
                               float(nu), int(nsteps), ctypes.c_void_p(buf.data_ptr()),
                               buf.numel(), _stream_ptr(stream),
                               ctypes.byref(st) if st is not None else None))
    if stats:
        return {f: getattr(st, f) for f, _ in StepStats._fields_}
    return rc


def frkc2_step_noalloc(grid, w, D=None, T=0.0, cfl=0.0, s=16, nu=0.01, nsteps=1, stream=None,
                       stats=False):
    """frkc2_step on the library's static scratch: no workspace, no device allocation."""
    lib = load()
    g = make_grid(grid)
    st = StepStats() if stats else None
    rc = _check(lib.frkc2_step_noalloc(ctypes.byref(g), _ptr(w), _ptr(D), float(T), float(cfl),
                                       int(s), float(nu), int(nsteps), _stream_ptr(stream),
                                       ctypes.byref(st) if st is not None else None))
    if stats:
        return {f: getattr(st, f) for f, _ in StepStats._fields_}
    return rc


def frkc2_integrate(grid, w, D=None, t_span=1.0, T0=1e-6, tol=1e-4, nu=0.01, max_attempts=10000,
                    trace_cap=0, stream=None, ws=None):
    """Error-controlled integration of w over t_span (in place). Returns (stats dict, trace),
    trace an array of (t, T, s, err, accepted) rows for the first trace_cap attempts."""
    lib = load()
    g = make_grid(grid)
    need = lib.frkc2_workspace_bytes(ctypes.byref(g), 0, WS_ADAPT)
    if need == 0:
        _check(-1)
    buf = ws if ws is not None else workspace(need, key="adapt")
    tr = np.zeros((max(int(trace_cap), 0), 5), dtype=np.float64)
    st = AdaptStats()
    _check(lib.frkc2_integrate(ctypes.byref(g), _ptr(w), _ptr(D), float(t_span), float(T0),
                               float(tol), float(nu), int(max_attempts),
                               ctypes.c_void_p(buf.data_ptr()), buf.numel(), _stream_ptr(stream),
                               tr.ctypes.data_as(_DP) if trace_cap > 0 else None, int(trace_cap),
                               ctypes.byref(st)))
    stats = {f: getattr(st, f) for f, _ in AdaptStats._fields_}
    return stats, tr[:min(stats["attempts"], tr.shape[0])]


def _user_views(buf, n):
    """Complex views into the workspace for the pointers the library passes to f."""
    torch = _torch()
    base = buf.data_ptr()
    cache = {}

    def view(ptr):
        off = int(ptr) - base
        if off < 0 or off + 16 * n > buf.numel() or off % 16:
            raise ValueError("stage pointer outside the workspace")
        if off not in cache:
            cache[off] = buf[off: off + 16 * n].view(torch.float64).view(torch.complex128)
        return cache[off]
    return view


def frkc2_step_user(w, f, T, rho=0.0, s=16, nu=0.01, nsteps=1, stream=None):
    """nsteps supersteps of w (float64, device) under a caller operator: f(W, F) receives the
    complex128 stage W and must write f(W) into F (both views of the library's workspace),
    on the current stream. The library applies the stepsizes and the Euler updates."""
    lib = load()
    n = int(w.numel())
    need = lib.frkc2_user_workspace_bytes(n, WS_STEP)
    if need == 0:
        _check(-1)
    buf = workspace(need, key="user")
    view = _user_views(buf, n)
    err = []

    def cb(W, F, nn, user, st):
        try:
            if nn != n:
                return 2
            f(view(W), view(F))
            return 0
        except Exception as e:   # reported after the call returns
            err.append(e)
            return 1

    cfun = USER_F(cb)
    rc = lib.frkc2_step_user(n, _ptr(w), cfun, None, float(T), float(rho), int(s), float(nu),
                             int(nsteps), ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                             _stream_ptr(stream))
    if err:
        raise err[0]
    return _check(rc)


def frkc2_integrate_user(w, f, rho, t_span, T0, tol, nu=0.01, max_attempts=100000, trace_cap=0,
                         stream=None):
    """Error-controlled integration of w (float64, device, in place) over t_span under a caller
    operator f(W, F) as in frkc2_step_user. rho is a spectral-radius bound of f's Jacobian: a
    number, or a function of the current state w (the caller's tensor) returning one, called
    before the first attempt and after every accepted step. Returns (stats dict, trace)."""
    lib = load()
    n = int(w.numel())
    need = lib.frkc2_user_workspace_bytes(n, WS_ADAPT)
    if need == 0:
        _check(-1)
    buf = workspace(need, key="user_adapt")
    view = _user_views(buf, n)
    err = []

    def cb(W, F, nn, user, st):
        try:
            if nn != n:
                return 2
            f(view(W), view(F))
            return 0
        except Exception as e:
            err.append(e)
            return 1

    def rcb(wp, nn, user, st, out):
        try:
            if nn != n or int(wp) != w.data_ptr():
                return 2
            out[0] = float(rho(w))
            return 0
        except Exception as e:
            err.append(e)
            return 1

    cfun = USER_F(cb)
    rfun = USER_RHO(rcb) if callable(rho) else ctypes.cast(None, USER_RHO)
    rho_const = 0.0 if callable(rho) else float(rho)
    tr = np.zeros((max(int(trace_cap), 0), 5), dtype=np.float64)
    st = AdaptStats()
    rc = lib.frkc2_integrate_user(n, _ptr(w), cfun, rfun, rho_const, None, float(t_span),
                                  float(T0), float(tol), float(nu), int(max_attempts),
                                  ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                  _stream_ptr(stream),
                                  tr.ctypes.data_as(_DP) if trace_cap > 0 else None,
                                  int(trace_cap), ctypes.byref(st))
    if err:
        raise err[0]
    _check(rc)
    stats = {f: getattr(st, f) for f, _ in AdaptStats._fields_}
    return stats, tr[:min(stats["attempts"], tr.shape[0])]


def frkc2_autotune(grid, w, D=None, s=16, nu=0.01, reps=2, stream=None, ws=None):
    """Time the pass configurations of frkc2_step on this grid and keep the fastest for it.
    w and D are only read. Returns the result fields as a dict."""
    lib = load()
    g = make_grid(grid)
    need = lib.frkc2_workspace_bytes(ctypes.byref(g), int(s), WS_STEP)
    if need == 0:
        _check(-1)
    buf = ws if ws is not None else workspace(need)
    r = TuneResult()
    _check(lib.frkc2_autotune(ctypes.byref(g), _ptr(w), _ptr(D), int(s), float(nu), int(reps),
                              ctypes.c_void_p(buf.data_ptr()), buf.numel(), _stream_ptr(stream),
                              ctypes.byref(r)))
    return {f: getattr(r, f) for f, _ in TuneResult._fields_}


def frkc2_step_adjoint(grid, w_n, D, T, s, lam_next, lam_n, grad_logD=None, nu=0.01,
                       stream=None, ws=None):
    lib = load()
    g = make_grid(grid)
    need = lib.frkc2_workspace_bytes(ctypes.byref(g), int(s), WS_ADJOINT)
    if need == 0:
        _check(-1)
    buf = ws if ws is not None else workspace(need, key="adjoint")
    return _check(lib.frkc2_step_adjoint(ctypes.byref(g), _ptr(w_n), _ptr(D), float(T), int(s),
                                         float(nu), _ptr(lam_next), _ptr(lam_n), _ptr(grad_logD),
                                         ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                         _stream_ptr(stream)))


def _store_ptr(t):
    """Pointer and byte size of a contiguous device buffer (the stage store)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or not t.is_contiguous():
        raise TypeError("expected a contiguous GPU tensor for the stage store")
    return ctypes.c_void_p(t.data_ptr()), t.numel() * t.element_size()


def stage_store(grid, s, device=None):
    """A new device buffer for one superstep's stage store (frkc2_step_store)."""
    torch = _torch()
    need = frkc2_workspace_bytes(grid, s, WS_STAGES)
    if need == 0:
        _check(-1)
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    return torch.empty(need, dtype=torch.uint8, device=dev)


def frkc2_step_store(grid, w, D, T, s, stages, nu=0.01, stream=None, ws=None):
    """One superstep in place on w that keeps its s stage states in stages."""
    lib = load()
    g = make_grid(grid)
    buf = ws if ws is not None else workspace(64 * 1024)
    sp, sb = _store_ptr(stages)
    return _check(lib.frkc2_step_store(ctypes.byref(g), _ptr(w), _ptr(D), float(T), int(s),
                                       float(nu), sp, sb, ctypes.c_void_p(buf.data_ptr()),
                                       buf.numel(), _stream_ptr(stream)))


def frkc2_step_adjoint_stored(grid, stages, D, T, s, lam_next, lam_n, grad_logD=None, nu=0.01,
                              stream=None, ws=None):
    lib = load()
    g = make_grid(grid)
    need = lib.frkc2_workspace_bytes(ctypes.byref(g), int(s), WS_ADJOINT_STORED)
    if need == 0:
        _check(-1)
    buf = ws if ws is not None else workspace(need, key="adjoint_stored")
    sp, sb = _store_ptr(stages)
    return _check(lib.frkc2_step_adjoint_stored(ctypes.byref(g), sp, sb, _ptr(D), float(T), int(s),
                                                float(nu), _ptr(lam_next), _ptr(lam_n),
                                                _ptr(grad_logD), ctypes.c_void_p(buf.data_ptr()),
                                                buf.numel(), _stream_ptr(stream)))


def frkc2_batched_workspace_bytes(grids, s_list) -> int:
    lib = load()
    n = len(grids)
    garr = (Grid * n)(*[make_grid(g) for g in grids])
    sarr = (ctypes.c_int * n)(*[int(v) for v in s_list])
    return int(lib.frkc2_batched_workspace_bytes(n, garr, sarr))


class BatchedArgs:
    """Marshalled arguments of one problem set (kept alive across graph replays)."""

    def __init__(self, grids, ws_list, D_list, T_list, s_list):
        n = len(grids)
        self.n = n
        self.grids = (Grid * n)(*[make_grid(g) for g in grids])
        self.w = (_VP * n)(*[_ptr(t) for t in ws_list])
        self.D = (_VP * n)(*[_ptr(t) if t is not None else None for t in D_list])
        self.T = (ctypes.c_double * n)(*[float(v) for v in T_list])
        self.s = (ctypes.c_int * n)(*[int(v) for v in s_list])
        self.tensors = (list(ws_list), list(D_list))


def frkc2_step_batched(args: BatchedArgs, nu=0.01, stream=None, ws=None):
    lib = load()
    need = lib.frkc2_batched_workspace_bytes(args.n, args.grids, args.s)
    if need == 0:
        _check(-1)
    buf = ws if ws is not None else workspace(need, key="batched")
    return _check(lib.frkc2_step_batched(args.n, args.grids, args.w, args.D, args.T, args.s,
                                         float(nu), ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                         _stream_ptr(stream)))


def frkc2_batched_autotune(args: BatchedArgs, nu=0.01, reps=2, stream=None, ws=None):
    """Time the batch's launch configurations on this problem set and keep the fastest for it.
    Every timed superstep advances the states in args (pass copies to keep them). Returns the
    result fields as a dict."""
    lib = load()
    need = lib.frkc2_batched_workspace_bytes(args.n, args.grids, args.s)
    if need == 0:
        _check(-1)
    buf = ws if ws is not None else workspace(need, key="batched")
    r = BatchTuneResult()
    _check(lib.frkc2_batched_autotune(args.n, args.grids, args.w, args.D, args.T, args.s,
                                      float(nu), int(reps), ctypes.c_void_p(buf.data_ptr()),
                                      buf.numel(), _stream_ptr(stream), ctypes.byref(r)))
    return {f: getattr(r, f) for f, _ in BatchTuneResult._fields_}


def frkc2_batched_config(grids, s_list):
    """(k3, cols3, k2) a graph built now for this problem set would use (host only)."""
    lib = load()
    n = len(grids)
    garr = (Grid * n)(*[make_grid(g) for g in grids])
    sarr = (ctypes.c_int * n)(*[int(v) for v in s_list])
    k3, c3, k2 = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib.frkc2_batched_config(n, garr, sarr, ctypes.byref(k3), ctypes.byref(c3),
                                    ctypes.byref(k2)))
    return k3.value, c3.value, k2.value


def frkc2_batched_status(ws=None, stream=None):
    buf = ws if ws is not None else workspace(0, key="batched")
    return _check(load().frkc2_batched_status(ctypes.c_void_p(buf.data_ptr()), _stream_ptr(stream)))


def frkc2_batched_release(ws=None):
    buf = ws if ws is not None else _ws_cache.get((_torch().cuda.current_device(), "batched"))
    if buf is None:
        return 0
    return _check(load().frkc2_batched_release(ctypes.c_void_p(buf.data_ptr())))


def frkc2_reduce(op: int, x, y=None, stream=None) -> float:
    lib = load()
    ws = workspace(64 * 1024)
    out = ctypes.c_double()
    _check(lib.frkc2_reduce(int(op), _ptr(x), _ptr(y), x.numel(), ctypes.byref(out),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    return out.value


def frkc2_write_table(path, nu: float = 0.01, m_max: int = 257):
    """Write the stepsize table (betabar, Q / Re a / Im a per M) in the public-code layout."""
    return _check(load().frkc2_write_table(os.fsencode(path), float(nu), int(m_max)))


def frkc2_stream_copy(src, dst, blocks_per_cu=4, nontemporal=False, stream=None):
    """Streaming copy of src into dst (device tensors of equal byte size), the HBM ceiling."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst sizes differ")
    return _check(load().frkc2_stream_copy(ctypes.c_void_p(src.data_ptr()),
                                           ctypes.c_void_p(dst.data_ptr()), nbytes,
                                           int(blocks_per_cu), int(bool(nontemporal)),
                                           _stream_ptr(stream)))


def frkc2_set_option(key: int, value: int):
    return _check(load().frkc2_set_option(int(key), int(value)))


def frkc2_last_error() -> str:
    return load().frkc2_last_error().decode()


def frkc2_version() -> str:
    return load().frkc2_version().decode()
