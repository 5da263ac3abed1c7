"""Oracle for the fourth-order split scheme FRKC4s (Sec. 4.1, "Complex splitting").

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module. The product library computes the same quantities in
its own code; the two share nothing but the numbers they print.

O'Sullivan, "Factorized Runge-Kutta-Chebyshev Methods" (arXiv:1702.03818):

* Sec. 4.1: for a reaction-diffusion system w' = A w + f_B(w) the scheme is a product of
  exponentials with complex time steps, B flows (the reaction, integrated on its own)
  alternating with A flows (the linear diffusion), starting and ending with a B flow.
  The paper points to the splitting literature for the coefficients and prints none.
* Sec. 2: the A flows are linear, so the FRKC polynomial of order N = 4,
  B(z) = d0 + 2 sum_{k=1..4} d_k C_{kM}(z), L = 4M, applied as L forward Euler steps
  with stepsizes a_l = 1 / (M^2 alpha_M (1 - zeta_l)) from its roots, is fourth-order
  accurate for them; the d_k follow from the linear order conditions R^(n)(0) = 1,
  n = 1..4.
* Sec. 2.2: the same internal-stability ordering as for N = 2.

Readings (each listed in the design doc):

* N = 4 polynomial. Write R(x) = P(C_M(z)) / P(1), z = 1 + x / (M^2 alpha_M), P of
  degree 4 in y = C_M(z) (so d0 + 2 sum d_k C_k(y) = P(y)). With g(x) = C_M(z(x)) the
  four order conditions fix the derivatives p_k = P^(k)(1) / P(1), k = 1..4, for any
  alpha_M (Faa di Bruno on P(g(x)) with g^(n)(0) = C_M^(n)(1) / (M^2 alpha_M)^n,
  C_M^(n)(1) = prod_{j<n} (M^2 - j^2) / (2j + 1)). Every x in [-2 M^2 alpha_M, 0] maps to
  y in [-1, 1], so |R| <= 1 there iff |P| <= 1 on [-1, 1]; the extent grows with alpha_M
  until P(-1) reaches 1 (P stays above its positive interior minimum elsewhere). N = 2
  under the same construction gives alpha_M = (4 - 1/M^2)/3, the closed form of the
  FRKC2 polynomial, and M = 1 gives the Taylor polynomial of e^x (classical RK4).
* Damping for N = 4 (Sec. 2.1 gives the mu-form; taken here as its effect): alpha_M is
  the value with P(-1) = 1 - nu0, nu0 = N nu, so the marginally stable real-axis points
  (C_M(z) = -1) have |R| = 1 - nu0; the extent shrinks by about one percent at
  nu = 0.01.
* Stage order: the roots y of P come in two conjugate pairs; the 2M stepsizes from the
  two roots with Im y > 0 are ordered greedily (as for N = 2, on L samples of
  [-betabar, 0]) and followed by their conjugates in the same order.
* Splitting: w^{n+1} = Re[ e^{b1 T B} e^{T/4 A} e^{b2 T B} e^{T/4 A} e^{b3 T B}
  e^{T/4 A} e^{b2 T B} e^{T/4 A} e^{b1 T B} w^n ], a symmetric composition with four
  equal real A steps (so every A flow uses the same real step and one stage table) and
  complex B steps. Symmetry gives the even orders; consistency and the two third-order
  conditions (the coefficients of [A,[A,B]] and [B,[B,A]]) leave exactly the conjugate
  pair b1 = (3 + i)/30, b2 = (4 - 2i)/15, b3 = (4 + 3i)/15 (and its conjugate), all with
  positive real parts; the real part is kept at the end of each step.
* B flows: dW/ds = tau f_B(W), s in [0, 1], along the complex time tau = b T, by nsub
  classical Runge-Kutta steps in s (f_B holomorphic); A flows: one FRKC4 superstep of
  length T/4 on the complex state.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import mpmath as mp
import numpy as np

from .coeffs import (N_SHRINK_MAX, SHRINK_C, _to_double, greedy_order, realised_q,
                     real_extent)

DPS = 50
S4_MAX = 512          # s = 4M, M <= 128


def cm_derivs(M: int, n: int):
    """C_M^(k)(1) for k = 1..n: prod_{j<k} (M^2 - j^2) / (2j + 1)."""
    out = []
    v = mp.mpf(1)
    for j in range(n):
        v = v * (mp.mpf(M) ** 2 - j * j) / (2 * j + 1)
        out.append(v)
    return out


def taylor_p(M: int, alpha, N: int = 4):
    """p_k = P^(k)(1)/P(1), k = 1..N, from R^(n)(0) = 1 (Faa di Bruno, N <= 4)."""
    c = cm_derivs(M, N)
    s = mp.mpf(M) ** 2 * alpha
    g = [c[k] / s ** (k + 1) for k in range(N)]   # g1..gN
    g1 = g[0]
    p1 = 1 / g1
    p = [p1]
    if N >= 2:
        p2 = (1 - p1 * g[1]) / g1 ** 2
        p.append(p2)
    if N >= 3:
        p3 = (1 - 3 * p2 * g1 * g[1] - p1 * g[2]) / g1 ** 3
        p.append(p3)
    if N >= 4:
        p4 = (1 - 6 * p3 * g1 ** 2 * g[1] - p2 * (3 * g[1] ** 2 + 4 * g1 * g[2])
              - p1 * g[3]) / g1 ** 4
        p.append(p4)
    return p


def p_value(M: int, alpha, y, N: int = 4):
    """P(y) with P(1) = 1 and the derivatives of taylor_p."""
    p = taylor_p(M, alpha, N)
    v = mp.mpf(1)
    f = mp.mpf(1)
    for k, pk in enumerate(p, 1):
        f *= k
        v += pk * (y - 1) ** k / f
    return v


def alpha_m(M: int, nu: float, N: int = 4):
    """The scale alpha_M with P(-1) = 1 - N nu, by bisection on [0.5, 3] (P(-1) increases
    with alpha_M across it)."""
    with mp.workdps(DPS):
        target = 1 - N * mp.mpf(nu)
        lo, hi = mp.mpf("0.5"), mp.mpf(3)
        f = lambda a: p_value(M, a, -1, N) - target
        if not (f(lo) < 0 < f(hi)):
            raise RuntimeError("alpha bracket")
        for _ in range(200):
            mid = (lo + hi) / 2
            if f(mid) < 0:
                lo = mid
            else:
                hi = mid
        return (lo + hi) / 2


def half_group(M: int, nu: float):
    """Stepsizes from the two roots y of P with Im y > 0 (2M mpc values), alpha_M, roots."""
    with mp.workdps(DPS):
        alpha = alpha_m(M, nu)
        p = taylor_p(M, alpha)
        # P(y) = 1 + sum p_k (y - 1)^k / k!  in powers of y (highest first)
        coef = [mp.mpf(0)] * 5
        coef[0] = mp.mpf(1)
        f = mp.mpf(1)
        for k, pk in enumerate(p, 1):
            f *= k
            for j in range(k + 1):
                coef[j] += pk / f * mp.binomial(k, j) * (-1) ** (k - j)
        ys = mp.polyroots(coef[::-1], maxsteps=400, extraprec=200)
        upper = sorted([y for y in ys if mp.im(y) > 0], key=lambda y: (mp.re(y), mp.im(y)))
        if len(upper) != 2:
            raise RuntimeError("expected two roots in the upper half plane")
        a = []
        for y in upper:
            th0 = mp.acos(y)
            for j in range(M):
                th = (th0 + 2 * mp.pi * j) / M
                one_minus = 2 * mp.sin(th / 2) ** 2
                a.append(1 / (mp.mpf(M) ** 2 * alpha * one_minus))
        return a, alpha, ys


@dataclass
class Coeffs4:
    a_re: np.ndarray
    a_im: np.ndarray
    beta: float
    beta_bar: float
    q_realised: float
    alpha: float
    n_shrink: int
    q_bound_met: bool

    @property
    def a(self) -> np.ndarray:
        return self.a_re + 1j * self.a_im


def frkc4_coeffs(s: int, nu: float = 0.01) -> Coeffs4:
    """Ordered stepsizes of the N = 4 FRKC polynomial (s = 4M stages) with beta, betabar,
    Q and n (Sec. 2 and 2.2; readings above)."""
    if s % 4 or s < 4 or s > S4_MAX:
        raise ValueError("s must be a multiple of 4, 4 <= s <= 512")
    if not (0.0 <= nu < 0.25):
        raise ValueError("nu must lie in [0, 0.25)")
    M = s // 4
    L = s
    a_h, alpha, _ = half_group(M, nu)
    ar = np.array([_to_double(mp.re(v)) for v in a_h])
    ai = np.array([_to_double(mp.im(v)) for v in a_h])
    beta0 = 2.0 * M * M * float(alpha)
    beta = real_extent(ar, ai, L, beta0)
    bound = 10.0 * L * L
    best = None
    for n in range(1, N_SHRINK_MAX + 1):
        beta_bar = (1.0 - n * SHRINK_C) * beta
        order = greedy_order(ar, ai, beta_bar, L)
        g = ar[order] + 1j * ai[order]
        seq = np.concatenate([g, np.conj(g)])
        q = realised_q(seq, beta, L)
        if best is None or q < best[0]:
            best = (q, n, beta_bar, seq)
        if q <= bound:
            break
    q, n, beta_bar, seq = best
    return Coeffs4(a_re=seq.real.copy(), a_im=seq.imag.copy(), beta=beta, beta_bar=beta_bar,
                   q_realised=q, alpha=float(alpha), n_shrink=n, q_bound_met=q <= bound)


# ---- the splitting (Sec. 4.1) ----

# B steps of the symmetric composition (exact rationals): b1, b2, b3, b2, b1
SPLIT_B = [(Fraction(3, 30), Fraction(1, 30)), (Fraction(4, 15), Fraction(-2, 15)),
           (Fraction(4, 15), Fraction(3, 15)), (Fraction(4, 15), Fraction(-2, 15)),
           (Fraction(3, 30), Fraction(1, 30))]
SPLIT_A = Fraction(1, 4)


def split_b():
    """The five B steps as complex doubles."""
    return [complex(float(r), float(i)) for r, i in SPLIT_B]


def split_sequence():
    """The composition as (operator, coefficient) from the first flow applied to the last."""
    out = []
    for j, b in enumerate(split_b()):
        out.append(("B", b))
        if j < 4:
            out.append(("A", float(SPLIT_A)))
    return out


def split_sequence_exact():
    """The composition with exact rational coefficients ((re, im) Fractions)."""
    out = []
    for j, b in enumerate(SPLIT_B):
        out.append(("B", b))
        if j < 4:
            out.append(("A", (SPLIT_A, Fraction(0))))
    return out


def react_flow_taus(b: complex, T: float, nsub: int):
    """Per-substep complex constants of a B flow: c = b T / nsub, c/2, c/6 (each as (re, im),
    formed in this order in FP64: tau = (Re b * T, Im b * T), c = tau / nsub, then halves and
    sixths of c)."""
    tr, ti = b.real * T, b.imag * T
    cr, ci = tr / nsub, ti / nsub
    return (cr, ci), (cr / 2.0, ci / 2.0), (cr / 6.0, ci / 6.0)


def a_stages(prob, T: float, s: int, nu: float = 0.01, coeffs: Coeffs4 | None = None):
    """Stepsizes tau_l = (T/4) a_l of one A flow (execution order)."""
    c = coeffs if coeffs is not None else frkc4_coeffs(s, nu)
    TA = T * float(SPLIT_A)
    return TA * c.a_re, TA * c.a_im


def step(prob, w, T: float, s: int, nsub: int = 4, nu: float = 0.01, coeffs=None):
    """One FRKC4s step of the two-species Brusselator (reaction B, diffusion A = d lap per
    species) from the real state w (v then w, 2N values). Returns the real state."""
    from . import stage
    N = prob.npoints
    zr = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(-1)).copy()
    zi = np.zeros_like(zr)
    tr, ti = a_stages(prob, T, s, nu, coeffs)
    for op, c in split_sequence():
        if op == "B":
            stage.react_flow(N, zr, zi, react_flow_taus(c, T, nsub), nsub)
        else:
            for sp in range(2):
                sl = slice(sp * N, (sp + 1) * N)
                r, i = zr[sl].copy(), zi[sl].copy()
                stage.superstep_complex(prob, r, i, tr, ti, op=0)
                zr[sl], zi[sl] = r, i
    return zr


def run(prob, T: float, s: int, nsteps: int, nsub: int = 4, nu: float = 0.01, w=None):
    c = frkc4_coeffs(s, nu)
    cur = np.asarray(prob.w0 if w is None else w, dtype=np.float64).reshape(-1).copy()
    for _ in range(nsteps):
        cur = step(prob, cur, T, s, nsub, nu, c)
    return cur
