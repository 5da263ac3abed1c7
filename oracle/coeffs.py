"""Oracle for the FRKC2 stepsizes: roots, damping, real extent and stage order.

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module. The product library computes the same
quantities in its own code; the two share nothing but the numbers they print.

Everything below follows O'Sullivan, "Factorized Runge-Kutta-Chebyshev Methods"
(arXiv:1702.03818):

* Sec. 2, "FRKC stability polynomials": the N = 2 polynomial is a sum of
  Chebyshev polynomials, B(z) = d0 + 2 d1 C_M(z) + 2 d2 C_2M(z) with L = 2M, the
  stepsizes come from its roots zeta_l as a_l = 1/(M^2 alpha_M) * 1/(1 - zeta_l),
  and the linear order conditions R'(0) = R''(0) = 1 fix the d_k.
* Sec. 2.1, "Damping": a_l = (1 - mu_l) / ((1 - nu) M^2 alpha_M (1 - (1 - 2 mu_l) zeta_l)),
  with N = 2 distinct mu values each repeated M times, found by Newton-Raphson
  on the order conditions.
* Sec. 2.2, "Internal stability": the amplification factors
  Q_jk(x) = prod_{l=j..k} |1 + a_l x|, the greedy ordering on the estimate
  Qbar over L sample points of [-betabar, 0], betabar = (1 - nC) beta, C = 1e-4,
  and the practical bound Q <= 10 L^2 that decides when n is incremented.

Closed form used for N = 2 (derived, not printed in the paper).  Write
R(x) = P(C_M(z)) / P(1) with z = 1 + x / (M^2 alpha_M) and P(y) = d0 + 2 d1 y +
2 d2 C_2(y).  The order conditions give R'(0) = P'(1) / alpha_M = 1 and
P''(1) + P'(1) (1 - 1/M^2)/3 = alpha_M^2 (P(1) = 1).  |P(-1)| <= 1 then forces
alpha_M <= 1 + (1 - 1/M^2)/3, and the bound is reached with d1 = 0, so the
extent-maximising choice is alpha_M = (4 - 1/M^2)/3, M^2 alpha_M = (L^2 - 1)/3,
and B is proportional to c0 + C_L(z) with c0 = (2L^2 + 1)/(L^2 - 1).  Its roots
are zeta_j = cos(theta_j), theta_j = (pi (2j+1) + i eta)/L, eta = arccosh(c0),
j = 0..L-1.  The undamped extent is beta0 = 2 M^2 alpha_M = 2 (L^2 - 1)/3.

Readings where the paper is silent or garbled (each is listed in the design doc):
* the M roots with C_M(zeta) = +i sinh(eta/2) (odd j) carry mu, the other M
  carry conj(mu), and the second group is built as exact conjugates of the
  first, so that every imaginary part cancels in the sum of the stages;
* the greedy ordering runs over the first group only (the product in Qbar
  stops at L/2) and the stage sequence is that order followed by the
  conjugates in the same order;
* the L sample points are x_k = -betabar k / L, k = 1..L;
* beta is the true real-axis extent of the damped polynomial built from the
  FP64 stepsizes (largest double b with |R(-x)| <= 1 on [0, b]);
* the realised Q is measured on max(4000, 10 L) evenly spaced points of
  [-beta, 0]; n runs from 1 to 64, and if no n meets the bound the order with
  the smallest Q is kept and flagged.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import mpmath as mp
import numpy as np
from mpmath import libmp

DPS = 50            # working precision of the root and damping computation
SHRINK_C = 1e-4     # C of Sec. 2.2
N_SHRINK_MAX = 64   # last n tried before giving up on Q <= 10 L^2
TIE_REL = 1e-12     # two greedy scores closer than this are a tie (lowest j wins)
S_MAX = 514         # M <= 257 (Sec. 3.1)


def _to_double(x) -> float:
    """Round an mpf to the nearest double (round-half-even)."""
    return libmp.to_float(mp.mpf(x)._mpf_, rnd="n")


@dataclass
class Coeffs:
    a_re: np.ndarray      # s stepsizes in execution order (real parts)
    a_im: np.ndarray      # (imaginary parts)
    beta: float           # real extent of the damped polynomial
    beta_bar: float       # (1 - n C) beta
    q_realised: float     # max_x max_{j<=k} prod |1 + a_l x| on [-beta, 0]
    mu: complex           # damping parameter of the first root group
    n_shrink: int         # n of Sec. 2.2
    q_bound_met: bool     # q_realised <= 10 L^2
    newton_iters: int

    @property
    def a(self) -> np.ndarray:
        return self.a_re + 1j * self.a_im


def undamped_roots(L: int):
    """Roots zeta_j of c0 + C_L(z) and 1 - zeta_j, both as mpc (Sec. 2, closed form above).

    1 - zeta is evaluated as 2 sin^2(theta/2) so that the roots closest to
    z = 1 (the largest stepsizes) keep their relative accuracy.
    """
    with mp.workdps(DPS):
        L2 = mp.mpf(L) ** 2
        c0 = (2 * L2 + 1) / (L2 - 1)
        eta = mp.acosh(c0)
        zeta, one_minus = [], []
        for j in range(L):
            theta = (mp.pi * (2 * j + 1) + 1j * eta) / L
            zeta.append(mp.cos(theta))
            one_minus.append(2 * mp.sin(theta / 2) ** 2)
        return zeta, one_minus, eta


def damped_group(L: int, nu: float):
    """Stepsizes of the first root group (odd j) after damping, as mpc (Sec. 2.1).

    a_j(mu) = K (1 - mu) / ((1 - zeta_j) + 2 mu zeta_j), K = 3/((1 - nu)(L^2 - 1)).
    The second group uses conj(mu) on the conjugate roots, so over all L stages
    sum a = 2 Re sum_G a and sum a^2 = 2 Re sum_G a^2.  Newton-Raphson on the two
    real equations 2 Re sum_G a = 1 (R'(0) = 1) and Re sum_G a^2 = 0
    (R''(0) = (sum a)^2 - sum a^2 = 1), starting from mu = 0.
    """
    zeta, one_minus, _ = undamped_roots(L)
    idx = [j for j in range(L) if j % 2 == 1]
    with mp.workdps(DPS):
        K = 3 / ((1 - mp.mpf(nu)) * (mp.mpf(L) ** 2 - 1))
        z = [zeta[j] for j in idx]
        om = [one_minus[j] for j in idx]
        mu = mp.mpc(0)
        iters = 0
        for iters in range(1, 101):
            den = [om[i] + 2 * mu * z[i] for i in range(len(idx))]
            a = [K * (1 - mu) / den[i] for i in range(len(idx))]
            da = [-K * (1 + z[i]) / den[i] ** 2 for i in range(len(idx))]
            F = mp.fsum(a)
            G = mp.fsum([ai * ai for ai in a])
            Fp = mp.fsum(da)
            Gp = mp.fsum([2 * a[i] * da[i] for i in range(len(idx))])
            e1 = 2 * mp.re(F) - 1
            e2 = 2 * mp.re(G)
            # d Re H / d Re mu = Re H',  d Re H / d Im mu = -Im H'
            j11, j12 = 2 * mp.re(Fp), -2 * mp.im(Fp)
            j21, j22 = 2 * mp.re(Gp), -2 * mp.im(Gp)
            det = j11 * j22 - j12 * j21
            dp = (e1 * j22 - j12 * e2) / det
            dq = (j11 * e2 - j21 * e1) / det
            mu = mu - mp.mpc(dp, dq)
            if abs(dp) + abs(dq) <= mp.mpf(10) ** (-(DPS - 8)):
                break
        den = [om[i] + 2 * mu * z[i] for i in range(len(idx))]
        a = [K * (1 - mu) / den[i] for i in range(len(idx))]
    return a, mu, iters


def log_abs_R_half(ar: np.ndarray, ai: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_G log|1 + a x| over the first group, for each real x.

    For real x the second group contributes the same magnitudes, so
    log|R(x)| = 2 * this.  Summing logs avoids any internal amplification.
    """
    x = np.asarray(x, dtype=np.float64)
    re = 1.0 + ar[:, None] * x[None, :]
    im = ai[:, None] * x[None, :]
    return np.log(np.hypot(re, im)).sum(axis=0)


def _R_abs_hp(ar, ai, x: float):
    """|R(x)| in DPS-digit arithmetic from the FP64 stepsizes of the first group."""
    with mp.workdps(DPS):
        xm = mp.mpf(x)
        p = mp.mpf(1)
        for r, i in zip(ar, ai):
            p *= (1 + mp.mpf(float(r)) * xm) ** 2 + (mp.mpf(float(i)) * xm) ** 2
        return p


def real_extent(ar: np.ndarray, ai: np.ndarray, L: int, beta0: float | None = None) -> float:
    """Largest double b with |R(-x)| <= 1 on [0, b] (Sec. 2: extent beta).

    A scan in FP64 log-magnitudes, dense where C_L oscillates fastest (eight
    points per half-period in z, then a few points past z = -1), finds the first
    sample above 1; bisection on doubles with the DPS-digit predicate
    |R(-b)| <= 1 + 1e-20 then locates the crossing. beta0 is the extent the
    scan is laid out on (default: the undamped N = 2 extent 2 (L^2 - 1)/3).
    """
    if beta0 is None:
        beta0 = 2.0 * (L * L - 1) / 3.0
    ks = np.arange(1, 8 * L + 1)
    zs = np.cos(ks * np.pi / (8 * L))
    xs = list((zs - 1.0) * (beta0 / 2.0))
    xs += [-beta0 * (1.0 + 1e-3 * j) for j in range(1, 41)]
    xs += [-beta0 * (1.04 + 0.05 * j) for j in range(1, 21)]   # reached only past 1.04 beta0
    xs = np.array(xs)
    lr = 2.0 * log_abs_R_half(ar, ai, xs)
    bad = np.nonzero(lr > 1e-12)[0]
    if len(bad) == 0:
        raise RuntimeError("no end of the stability interval found")
    i = int(bad[0])
    lo = 0.0 if i == 0 else -float(xs[i - 1])
    hi = -float(xs[i])
    one = mp.mpf(1) + mp.mpf(10) ** -20

    def stable(b):
        return _R_abs_hp(ar, ai, -b) <= one

    while True:
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return lo


def greedy_order(ar: np.ndarray, ai: np.ndarray, beta_bar: float, L: int) -> list[int]:
    """Greedy stage order of the first group (Sec. 2.2, estimate Qbar).

    v_jk = |1 + a_j x_k| on x_k = -betabar k / L, k = 1..L.  With the product p_k
    of the stages already placed and the set S of stages not yet placed, the
    next stage is the c in S that minimises
        sum_k max(p_k v_ck, prod_{j in S, j != c} v_jk),
    i.e. the 1-norm over the samples of the larger of the prefix product up to
    and including c and the product of the stages that would remain after it.
    Scores are formed from log-magnitudes; a score within TIE_REL of the
    minimum counts as a tie and the lowest index wins.
    """
    M = len(ar)
    x = np.array([-(beta_bar * k) / L for k in range(1, L + 1)])
    lv = np.log(np.hypot(1.0 + ar[:, None] * x[None, :], ai[:, None] * x[None, :]))
    placed = np.zeros(L)
    S = list(range(M))
    order = []
    for _ in range(M):
        rest = lv[S].sum(axis=0)
        pre = placed[None, :] + lv[S]
        suf = rest[None, :] - lv[S]
        scores = np.exp(np.maximum(pre, suf)).sum(axis=1)
        m = scores.min()
        pick = next(i for i in range(len(S)) if scores[i] <= m * (1.0 + TIE_REL))
        c = S.pop(pick)
        order.append(c)
        placed = placed + lv[c]
    return order


def realised_q(a: np.ndarray, beta: float, L: int) -> float:
    """Q of Sec. 2.2: max over x in [-beta, 0] and all runs j <= k of prod |1 + a_l x|.

    The maximum over runs is Kadane's maximum-subarray scan of log|1 + a_l x|
    along the stage sequence, on max(4000, 10 L) evenly spaced x.
    """
    G = max(4000, 10 * L)
    x = np.linspace(-beta, 0.0, G)
    best = np.full(G, -np.inf)
    cur = np.zeros(G)
    for l in range(len(a)):
        t = np.log(np.abs(1.0 + a[l] * x))
        cur = np.maximum(t, cur + t)
        best = np.maximum(best, cur)
    return float(np.exp(best.max()))


def frkc2_coeffs(s: int, nu: float = 0.01) -> Coeffs:
    """Ordered FRKC2 stepsizes a_1..a_s (sum a = 1) with beta, betabar, Q and n."""
    if s % 2 or s < 2 or s > S_MAX:
        raise ValueError("s must be even, 2 <= s <= 514")
    if not (0.0 <= nu < 1.0):
        raise ValueError("nu must lie in [0, 1)")
    L = s
    a_g, mu, iters = damped_group(L, nu)
    ar = np.array([_to_double(mp.re(v)) for v in a_g])
    ai = np.array([_to_double(mp.im(v)) for v in a_g])
    beta = real_extent(ar, ai, L)
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
    return Coeffs(a_re=seq.real.copy(), a_im=seq.imag.copy(), beta=beta,
                  beta_bar=beta_bar, q_realised=q,
                  mu=complex(_to_double(mp.re(mu)), _to_double(mp.im(mu))),
                  n_shrink=n, q_bound_met=q <= bound, newton_iters=iters)


def stability_poly(a: np.ndarray, x) -> np.ndarray:
    """R(x) = prod_l (1 + a_l x) for complex x (Sec. 2, factorised form)."""
    x = np.asarray(x, dtype=np.complex128)
    r = np.ones_like(x)
    for al in a:
        r = r * (1.0 + al * x)
    return r
