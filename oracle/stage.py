"""ctypes wrapper of the plain C stage-loop oracle (stage.c).

TEST INFRASTRUCTURE: imported only by the tests, the smoke check and the
CPU-baseline leg of the benchmark.

The wrapper only marshals arrays. The stepsizes tau_l = T a_l are formed here
in FP64 from the oracle's own coefficients, and T itself is either given or,
for the adaptive choice, (cfl * betabar) / rho with rho the Gershgorin bound of
the current state (the stability requirement T rho <= betabar of Sec. 2;
cfl < 1 is a safety factor, a proposed reading: the paper leaves the choice of
T to the user of its stepsize table).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .coeffs import frkc2_coeffs

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
# The same source with every fused multiply-add evaluated as a*b + c (two
# roundings): used only to measure how far the fused order moves results.
_LIB_UNFUSED = os.path.join(_HERE, "_build", "liboracle_unfused.so")
_lib = None
_lib_unfused = None


def build(force: bool = True) -> str:
    """Compile stage.c with gcc (FP64, no contraction, OpenMP over points), and its unfused
    variant."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    for path, extra in ((_LIB_PATH, []), (_LIB_UNFUSED, ["-DORACLE_UNFUSED"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                                   "-fopenmp", "-fPIC", "-shared"] + extra +
                                  ["-o", tmp, os.path.join(_HERE, "stage.c"), "-lm"])
            os.replace(tmp, path)
    return _LIB_PATH


def _load(unfused: bool = False):
    global _lib, _lib_unfused
    if unfused and _lib_unfused is None:
        _load()
        lib = ctypes.CDLL(_LIB_UNFUSED)
        _declare(lib)
        _lib_unfused = lib
    if unfused:
        return _lib_unfused
    if _lib is None:
        src = os.path.join(_HERE, "stage.c")
        stale = any(not os.path.exists(p) or os.path.getmtime(src) > os.path.getmtime(p)
                    for p in (_LIB_PATH, _LIB_UNFUSED))
        if stale:
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        _declare(lib)
        _lib = lib
    return _lib


def _declare(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_long)
    common = [ctypes.c_int, lp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
              dp, ctypes.c_int, dp, dp]
    lib.oracle_superstep.argtypes = common + [dp, dp, dp, dp]
    lib.oracle_superstep.restype = ctypes.c_int
    lib.oracle_adjoint.argtypes = common + [dp, dp, dp, dp]
    lib.oracle_adjoint.restype = ctypes.c_int
    lib.oracle_rho_bound.argtypes = [ctypes.c_int, lp, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, dp, dp]
    lib.oracle_rho_bound.restype = ctypes.c_double
    lib.oracle_set_faces.argtypes = [dp]
    lib.oracle_set_faces.restype = None
    lib.oracle_euler_update.argtypes = [ctypes.c_long, dp, dp, dp, dp, ctypes.c_double,
                                        ctypes.c_double, dp]
    lib.oracle_euler_update.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_superstep_c.argtypes = common + [dp, dp]
    lib.oracle_superstep_c.restype = ctypes.c_int
    lib.oracle_react_flow.argtypes = [ctypes.c_long, dp, dp] + [ctypes.c_double] * 6 + [ctypes.c_int]
    lib.oracle_react_flow.restype = None


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def face_coefficients(prob):
    """Op 4 (advection-diffusion, central differences): coefficient of face f = 2*dim + side,
    d + (0.5*h)*v_dim on the minus side and d - (0.5*h)*v_dim on the plus side."""
    vel = list(getattr(prob, "vel", (0.0, 0.0, 0.0))) + [0.0] * 3
    fc = np.empty(6)
    for k in range(3):
        fc[2 * k] = prob.d_const + (0.5 * prob.h) * vel[k]
        fc[2 * k + 1] = prob.d_const - (0.5 * prob.h) * vel[k]
    return fc


def _grid_args(prob, lib=None):
    n = (ctypes.c_long * 3)(*[int(v) for v in prob.n])
    inv_h2 = 1.0 / (prob.h * prob.h)
    lib = lib if lib is not None else _load()
    if prob.op == 4:
        _grid_args.fc = face_coefficients(prob)
        lib.oracle_set_faces(_dp(_grid_args.fc))
    else:
        lib.oracle_set_faces(None)
    return n, inv_h2


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64).reshape(-1)


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """OpenMP threads for the oracle's loops from now on."""
    _load().oracle_set_threads(int(n))


def superstep(prob, w, tau_re, tau_im, D=None, want_imag=False, unfused=False):
    """One superstep from real w with stepsizes tau (execution order). Returns Re W^s (and Im W^s).
    unfused=True runs the variant that rounds every multiply-add twice (a*b + c)."""
    lib = _load(unfused)
    n, inv_h2 = _grid_args(prob, lib)
    wr = _f64(w).copy()
    wi = np.empty_like(wr) if want_imag else None
    Dd = _f64(D if D is not None else prob.D) if (prob.D is not None or D is not None) else None
    tr, ti = _f64(tau_re), _f64(tau_im)
    rc = lib.oracle_superstep(prob.ndim, n, prob.bc, prob.op, inv_h2, prob.d_const, _dp(Dd),
                              len(tr), _dp(tr), _dp(ti), _dp(wr), _dp(wi), None, None)
    if rc != 0:
        raise RuntimeError("oracle_superstep failed (%d)" % rc)
    return (wr, wi) if want_imag else wr


def superstep_embedded(prob, w, tau_re, tau_im, D=None):
    """One superstep from real w that also carries the embedded first-order solution of
    Sec. 3 (real parts of the stepsizes and of f only). Returns (Re W^s, Im W^s, What^s)."""
    lib = _load()
    n, inv_h2 = _grid_args(prob)
    wr = _f64(w).copy()
    wi = np.empty_like(wr)
    wh = np.empty_like(wr)
    Dd = _f64(D if D is not None else prob.D) if (prob.D is not None or D is not None) else None
    tr, ti = _f64(tau_re), _f64(tau_im)
    rc = lib.oracle_superstep(prob.ndim, n, prob.bc, prob.op, inv_h2, prob.d_const, _dp(Dd),
                              len(tr), _dp(tr), _dp(ti), _dp(wr), _dp(wi), None, _dp(wh))
    if rc != 0:
        raise RuntimeError("oracle_superstep failed (%d)" % rc)
    return wr, wi, wh


def rho_bound(prob, w=None, D=None) -> float:
    """Gershgorin bound of f's Jacobian; the porous and Brusselator bounds depend on the
    state w (prob.w0 if w is None)."""
    lib = _load()
    n, inv_h2 = _grid_args(prob)
    Dd = D if D is not None else prob.D
    Dd = _f64(Dd) if Dd is not None else None
    if w is None and prob.op in (2, 3):
        w = prob.w0
    ww = _f64(w) if w is not None else None
    r = lib.oracle_rho_bound(prob.ndim, n, prob.bc, prob.op, inv_h2, prob.d_const,
                             _dp(Dd), _dp(ww))
    if r < 0:
        raise ValueError("rho_bound: invalid grid, or a state (porous, Brusselator) or D "
                         "(variable coefficient) missing")
    return r


def run(prob, s, nsteps, T=None, cfl=None, nu=0.01, w=None, coeffs=None):
    """nsteps supersteps of s stages; fixed T, or T = (cfl*betabar)/rho(w_n) per superstep.

    Returns (w, list of T used).
    """
    c = coeffs if coeffs is not None else frkc2_coeffs(s, nu)
    cur = _f64(prob.w0 if w is None else w).copy()
    Ts = []
    for _ in range(nsteps):
        if cfl is not None:
            Tn = (cfl * c.beta_bar) / rho_bound(prob, cur)
        else:
            Tn = float(T)
        Ts.append(Tn)
        cur = superstep(prob, cur, Tn * c.a_re, Tn * c.a_im)
    return cur, Ts


def adjoint(prob, w_n, lam_next, tau_re, tau_im, grad_logD=None, D=None, unfused=False):
    """Adjoint of one superstep: returns lam_n and grad_logD (accumulated in place).
    unfused=True runs the variant that rounds every multiply-add twice."""
    lib = _load(unfused)
    n, inv_h2 = _grid_args(prob, lib)
    Dd = D if D is not None else prob.D
    Dd = _f64(Dd) if Dd is not None else None
    wn = _f64(w_n)
    ln = _f64(lam_next)
    out = np.empty_like(wn)
    g = grad_logD if grad_logD is not None else np.zeros_like(wn)
    tr, ti = _f64(tau_re), _f64(tau_im)
    rc = lib.oracle_adjoint(prob.ndim, n, prob.bc, prob.op, inv_h2, prob.d_const, _dp(Dd),
                            len(tr), _dp(tr), _dp(ti), _dp(wn), _dp(ln), _dp(out), _dp(g))
    if rc != 0:
        raise RuntimeError("oracle_adjoint failed (%d)" % rc)
    return out, g


def euler_update(wr, wi, fr, fi, tr, ti, emb=None):
    """W <- W + tau f in place (wr, wi: contiguous float64), and emb <- emb + Re tau Re f."""
    for a in (wr, wi, fr, fi) + ((emb,) if emb is not None else ()):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    _load().oracle_euler_update(wr.size, _dp(wr), _dp(wi), _dp(fr), _dp(fi), float(tr), float(ti),
                                _dp(emb))


def superstep_complex(prob, wr, wi, tau_re, tau_im, op=None, D=None):
    """s stages on the complex state (wr, wi) in place (contiguous float64), the operator of
    prob (or op; op 0 with prob.d_const is the diffusion flow of the split scheme)."""
    lib = _load()
    n, inv_h2 = _grid_args(prob)
    for a in (wr, wi):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    opv = prob.op if op is None else op
    Dd = D if D is not None else (prob.D if opv == 1 else None)
    Dd = _f64(Dd) if Dd is not None else None
    tr, ti = _f64(tau_re), _f64(tau_im)
    rc = lib.oracle_superstep_c(prob.ndim, n, prob.bc, opv, inv_h2, prob.d_const, _dp(Dd),
                                len(tr), _dp(tr), _dp(ti), _dp(wr), _dp(wi))
    if rc != 0:
        raise RuntimeError("oracle_superstep_c failed (%d)" % rc)


def react_flow(N, zr, zi, taus, nsub):
    """Brusselator reaction flow over a complex time (in place; v then w in zr, zi); taus =
    (c, c/2, c/6) as (re, im) pairs, c = tau / nsub."""
    for a in (zr, zi):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"] and a.size == 2 * N
    (cr, ci), (c2r, c2i), (c6r, c6i) = taus
    _load().oracle_react_flow(int(N), _dp(zr), _dp(zi), cr, ci, c2r, c2i, c6r, c6i, int(nsub))
