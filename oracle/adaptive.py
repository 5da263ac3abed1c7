"""Error-controlled FRKC2 integration (O'Sullivan, arXiv:1702.03818, Sec. 3).

TEST INFRASTRUCTURE, like the rest of this package.

Sec. 3 gets an error estimate for free: besides the complex stages W^l, the
embedded first-order solution What uses only the real parts of the stepsizes
and of f(W^l) (oracle.stage.superstep_embedded). The scaled error is

    err = || |W^L - What^L| / (TOL (1 + max(|W^L|, |What^L|))) ||,

a step with err > 1 is retried with T scaled by SAFE / sqrt(err), and after an
accepted step the predictive controller

    T_next = T_n (SAFE / sqrt(err_n)) (T_n / T_{n-1}) sqrt(err_{n-1} / err_n)

sets the next length, with SAFE = 0.8.

Readings (the section leaves these open; the GPU library takes the same ones):
  * the norm is the maximum over grid points; |.| is the complex modulus, with
    |z| = sqrt(re*re + im*im) and each term evaluated without fused
    multiply-adds;
  * the printed controller is a ratio: it multiplies the current length T_n;
    it is used after two consecutive accepted steps, and the plain
    T_n SAFE / sqrt(err_n) otherwise; err values below 1e-12 count as 1e-12,
    and the growth factor is capped at 5;
  * each attempt takes the smallest even s whose betabar(s) covers T rho
    (rho the Gershgorin bound; for the porous operator and the Brusselator, of
    the current state),
    searched from s = 2 ceil(sqrt(T rho / 1.32)) downward and upward in steps
    of 2 (betabar ~ 0.33 s^2); if betabar(514) is too small, T is cut to
    0.99 betabar(514) / rho;
  * the last step is shortened to end exactly at t_span; the new state is
    Re W^L.
"""
import math

import numpy as np

from . import stage
from .coeffs import frkc2_coeffs

SAFE = 0.8
FACMAX = 5.0
ERR_FLOOR = 1e-12
S_MAX = 514

_coeff_cache = {}


def coeffs(s, nu):
    key = (s, nu)
    if key not in _coeff_cache:
        _coeff_cache[key] = frkc2_coeffs(s, nu)
    return _coeff_cache[key]


def choose_s(x, nu):
    """Smallest even s with betabar(s) >= x, searched from the quadratic estimate."""
    m = math.ceil(math.sqrt(x / 1.32))
    m = min(max(m, 1), S_MAX // 2)
    s = 2 * m
    while s > 2 and coeffs(s - 2, nu).beta_bar >= x:
        s -= 2
    while s < S_MAX and coeffs(s, nu).beta_bar < x:
        s += 2
    return s


def error_norm(wr, wi, wh, tol):
    """Max over points of |W - What| / (tol (1 + max(|W|, |What|))); NaN counts as inf."""
    dr = wr - wh
    num = np.sqrt(dr * dr + wi * wi)
    mw = np.sqrt(wr * wr + wi * wi)
    den = tol * (1.0 + np.maximum(mw, np.abs(wh)))
    e = num / den
    e = np.where(np.isnan(e), np.inf, e)
    return float(np.max(e))


def integrate(prob, t_span, T0, tol, nu=0.01, w=None, max_attempts=10000):
    """Advance the state by t_span with error control. Returns (w, trace, T_next) where trace
    lists (t, T, s, err, accepted) per attempt."""
    cur = np.ascontiguousarray(prob.w0 if w is None else w, dtype=np.float64).reshape(-1).copy()
    t = 0.0
    T = float(T0)
    have_prev = False
    T_prev = err_prev = 0.0
    rho = None
    trace = []
    while t < t_span:
        if len(trace) >= max_attempts:
            raise RuntimeError("attempt limit reached")
        if rho is None or prob.op in (2, 3):
            rho = stage.rho_bound(prob, cur)
        Tn = min(T, t_span - t)
        x = Tn * rho
        s = choose_s(x, nu)
        c = coeffs(s, nu)
        if c.beta_bar < x:
            Tn = 0.99 * c.beta_bar / rho
        wr, wi, wh = stage.superstep_embedded(prob, cur, Tn * c.a_re, Tn * c.a_im)
        err = error_norm(wr, wi, wh, tol)
        if not math.isfinite(err):
            raise FloatingPointError("non-finite error estimate")
        if err > 1.0:
            trace.append((t, Tn, s, err, 0))
            T = Tn * (SAFE / math.sqrt(err))
            have_prev = False
            continue
        trace.append((t, Tn, s, err, 1))
        cur = wr
        t = t + Tn
        e = max(err, ERR_FLOOR)
        fac = SAFE / math.sqrt(e)
        if have_prev:
            fac = fac * (Tn / T_prev) * math.sqrt(err_prev / e)
        fac = min(fac, FACMAX)
        T_prev = Tn
        err_prev = e
        have_prev = True
        T = Tn * fac
        if prob.op in (2, 3):
            rho = None
    return cur, trace, T


def superstep_user(f, w, tau_re, tau_im):
    """One superstep around a caller operator f(wr, wi) -> (fr, fi) (the core/user split of the
    paper's public code, Sec. 3.1), carrying the embedded solution. Returns (Wr, Wi, What)."""
    wr = np.ascontiguousarray(w, dtype=np.float64).reshape(-1).copy()
    wi = np.zeros_like(wr)
    emb = wr.copy()
    for tr, ti in zip(tau_re, tau_im):
        fr, fi = f(wr, wi)
        stage.euler_update(wr, wi, np.ascontiguousarray(fr, dtype=np.float64),
                           np.ascontiguousarray(fi, dtype=np.float64), tr, ti, emb)
    return wr, wi, emb


def integrate_user(f, rho, w0, t_span, T0, tol, nu=0.01, max_attempts=10000):
    """Error control of Sec. 3 (the readings above) around a caller operator f. rho is a
    spectral-radius bound: a number, or a function of the current real state, evaluated
    before the first attempt and after every accepted step. Returns (w, trace, T_next)."""
    cur = np.ascontiguousarray(w0, dtype=np.float64).reshape(-1).copy()
    t = 0.0
    T = float(T0)
    have_prev = False
    T_prev = err_prev = 0.0
    r = None
    trace = []
    while t < t_span:
        if len(trace) >= max_attempts:
            raise RuntimeError("attempt limit reached")
        if r is None:
            r = float(rho(cur)) if callable(rho) else float(rho)
        Tn = min(T, t_span - t)
        x = Tn * r
        s = choose_s(x, nu)
        c = coeffs(s, nu)
        if c.beta_bar < x:
            Tn = 0.99 * c.beta_bar / r
        wr, wi, wh = superstep_user(f, cur, Tn * c.a_re, Tn * c.a_im)
        err = error_norm(wr, wi, wh, tol)
        if not math.isfinite(err):
            raise FloatingPointError("non-finite error estimate")
        if err > 1.0:
            trace.append((t, Tn, s, err, 0))
            T = Tn * (SAFE / math.sqrt(err))
            have_prev = False
            continue
        trace.append((t, Tn, s, err, 1))
        cur = wr
        t = t + Tn
        e = max(err, ERR_FLOOR)
        fac = SAFE / math.sqrt(e)
        if have_prev:
            fac = fac * (Tn / T_prev) * math.sqrt(err_prev / e)
        fac = min(fac, FACMAX)
        T_prev = Tn
        err_prev = e
        have_prev = True
        T = Tn * fac
        if callable(rho):
            r = None
    return cur, trace, T
