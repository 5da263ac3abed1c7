"""Pins of the fourth-order oracle (Sec. 4.1 complex splitting with FRKC4 linear flows).

N = 4 polynomial: the four order conditions (elementary symmetric functions of the stepsizes),
the M = 1 special case (classical RK4, real extent 2.7853), the reduction of the same
construction to the FRKC2 closed form at N = 2, stability on [-beta, 0] by brute force, the
damped marginal points, maximality of the extent at nu = 0, the internal-stability bound.
Splitting: the order conditions in exact rational arithmetic up to degree 4, local error h^5 on
random matrices against scipy's expm. Reaction flow: Runge-Kutta order in nsub against scipy's
DOP853 in real and complex time. Whole scheme: fourth-order convergence on the Brusselator
against DOP853 on an independent numpy stencil.
"""
from fractions import Fraction
from math import factorial

import mpmath as mp
import numpy as np
import pytest

from oracle import frkc4, stage
from paper_1702_03818_amd import workloads as wl


def elem_sym(a, kmax=5):
    e = np.zeros(kmax + 1, dtype=complex)
    e[0] = 1.0
    for al in a:
        for k in range(kmax, 0, -1):
            e[k] += al * e[k - 1]
    return e


@pytest.mark.parametrize("s", [4, 8, 12, 16, 32, 64, 100, 128, 256])
def test_order_conditions(s):
    """R(x) = prod (1 + a_l x) = sum e_k x^k with e_k = 1/k! for k <= 4 (and not for k = 5)."""
    c = frkc4.frkc4_coeffs(s, 0.01)
    e = elem_sym(c.a)
    for k in range(1, 5):
        assert abs(e[k] - 1.0 / factorial(k)) <= 1e-12 * max(1.0, c.q_realised / s) / factorial(k)
    assert abs(e[5] - 1.0 / 120) > 1e-6


def test_rk4_special_case():
    """M = 1: the polynomial is the degree-4 Taylor polynomial of e^x (classical RK4) and its
    real extent is where |1 + x + x^2/2 + x^3/6 + x^4/24| = 1 first fails, 2.78529356..."""
    c = frkc4.frkc4_coeffs(4, 0.01)
    e = elem_sym(c.a)
    assert np.allclose(e[:5], [1, 1, 0.5, 1 / 6, 1 / 24], rtol=0, atol=1e-15)
    taylor = np.polynomial.Polynomial([1, 1, 0.5, 1 / 6, 1 / 24])
    r = (taylor - 1).roots()
    x = min(v.real for v in r if abs(v.imag) < 1e-9 and v.real < -1e-6)
    assert abs(c.beta - (-x)) <= 1e-12 * abs(x)
    assert abs(c.beta - 2.785293563405282) < 1e-12


@pytest.mark.parametrize("M", [1, 2, 3, 8, 50, 257])
def test_same_construction_gives_frkc2_at_n2(M):
    """With N = 2 the scale that puts P(-1) at 1 is alpha_M = (4 - 1/M^2)/3, the closed form
    of the second-order polynomial (an independent check of the order-condition algebra)."""
    with mp.workdps(50):
        a = frkc4.alpha_m(M, 0.0, N=2)
        assert abs(a - (4 - mp.mpf(1) / M ** 2) / 3) < mp.mpf(10) ** -40


@pytest.mark.parametrize("s,nu", [(8, 0.01), (32, 0.01), (64, 0.0), (100, 0.01), (256, 0.01)])
def test_stable_on_extent(s, nu):
    """|R| <= 1 on a dense grid of [-beta, 0]; > 1 a little beyond -beta."""
    c = frkc4.frkc4_coeffs(s, nu)
    x = np.linspace(-c.beta, 0.0, 200001)
    lg = np.zeros_like(x)
    for al in c.a:
        lg += np.log(np.abs(1.0 + al * x))
    assert lg.max() <= 1e-10
    xb = -c.beta * (1 + 1e-6)
    assert sum(np.log(np.abs(1.0 + al * xb)) for al in c.a) > 0


@pytest.mark.parametrize("M", [2, 5, 16, 64])
def test_damped_marginal_points(M):
    """Where C_M(z) = -1 inside [-beta, 0], |R| = P(-1) = 1 - 4 nu (Sec. 2.1's effect of
    damping: the marginally stable maxima are scaled by 1 - nu0)."""
    nu = 0.01
    c = frkc4.frkc4_coeffs(4 * M, nu)
    scale = M * M * c.alpha
    for j in range(M):
        z = np.cos((2 * j + 1) * np.pi / M)
        x = scale * (z - 1.0)
        R = np.prod(1.0 + c.a * x)
        assert abs(abs(R) - (1 - 4 * nu)) < 1e-9 * c.q_realised


@pytest.mark.parametrize("M", [2, 7, 32])
def test_extent_maximal_at_nu0(M):
    """At nu = 0 a slightly larger alpha_M breaks |P| <= 1 on [-1, 1]; the chosen one keeps it."""
    with mp.workdps(50):
        a = frkc4.alpha_m(M, 0.0)
        ys = [-1 + 2 * mp.mpf(i) / 2000 for i in range(2001)]
        assert max(abs(frkc4.p_value(M, a, y)) for y in ys) <= 1 + mp.mpf(10) ** -30
        a2 = a * (1 + mp.mpf(10) ** -6)
        assert max(abs(frkc4.p_value(M, a2, y)) for y in ys) > 1


def test_internal_stability_bound():
    """Q <= 10 L^2 (Sec. 2.2) with the greedy order; a natural order is far worse."""
    ns = []
    for s in range(8, 260, 8):
        c = frkc4.frkc4_coeffs(s, 0.01)
        assert c.q_bound_met and c.q_realised <= 10.0 * s * s
        ns.append(c.n_shrink)
    assert np.mean(ns) < 3
    a_h, _, _ = frkc4.half_group(64, 0.01)
    h = np.array([complex(v) for v in a_h])
    natural = np.concatenate([h, np.conj(h)])
    from oracle.coeffs import realised_q
    c = frkc4.frkc4_coeffs(256, 0.01)
    assert realised_q(natural, c.beta, 256) > 1e3 * c.q_realised


# ---- splitting ----

class G:
    """Gaussian rational: exact complex arithmetic on Fractions."""
    def __init__(self, re, im=0):
        self.re, self.im = Fraction(re), Fraction(im)

    def __add__(self, o):
        return G(self.re + o.re, self.im + o.im)

    def __mul__(self, o):
        return G(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def scale(self, f):
        return G(self.re * f, self.im * f)

    def __eq__(self, o):
        return self.re == o.re and self.im == o.im


def _mul(x, y, deg):
    out = {}
    for a, ca in x.items():
        for b, cb in y.items():
            w = a + b
            if len(w) <= deg:
                out[w] = out.get(w, G(0)) + ca * cb
    return out


def _exp(sym, c, deg):
    out, term = {"": G(1)}, {"": G(1)}
    for k in range(1, deg + 1):
        term = {w: v.scale(Fraction(1, k)) for w, v in _mul(term, {sym: c}, deg).items()}
        for w, v in term.items():
            out[w] = out.get(w, G(0)) + v
    return out


def test_split_order_conditions_exact():
    """In the free algebra of A and B, the composition with b = (3+i)/30, (4-2i)/15,
    (4+3i)/15, (4-2i)/15, (3+i)/30 and four A steps of 1/4 equals exp(A + B) in every word of
    length <= 4 (fourth order), exactly; some word of length 5 differs."""
    deg = 5
    comp = {"": G(1)}
    for op, c in frkc4.split_sequence_exact():
        comp = _mul(comp, _exp(op, G(*c), deg), deg)
    target, term = {"": G(1)}, {"": G(1)}
    for k in range(1, deg + 1):
        term = {w: v.scale(Fraction(1, k)) for w, v in _mul(term, {"A": G(1), "B": G(1)}, deg).items()}
        for w, v in term.items():
            target[w] = target.get(w, G(0)) + v
    words4 = [w for w in target if len(w) <= 4]
    assert all(comp.get(w, G(0)) == target[w] for w in words4)
    assert any(not (comp.get(w, G(0)) == target[w]) for w in target if len(w) == 5)
    assert all(b.real > 0 for b in frkc4.split_b())


def test_split_local_error_matrices():
    """Random matrices (A symmetric negative semi-definite, B general): the composition of
    matrix exponentials differs from expm(h (A + B)) by O(h^5)."""
    from scipy.linalg import expm
    rng = np.random.default_rng(3)
    X = rng.standard_normal((6, 6))
    A = -(X @ X.T) / 6
    B = rng.standard_normal((6, 6)) / 2
    errs = []
    for h in (0.2, 0.1, 0.05):
        P = np.eye(6, dtype=complex)
        for op, c in frkc4.split_sequence():
            P = expm(c * h * (A if op == "A" else B)) @ P
        errs.append(np.abs(P - expm(h * (A + B))).max())
    r = [errs[i] / errs[i + 1] for i in range(2)]
    assert 28 < r[-1] < 36


# ---- reaction flow ----

def _react(tau, y0, nsub):
    N = 1
    zr = np.array([y0[0].real, y0[1].real])
    zi = np.array([y0[0].imag, y0[1].imag])
    b = tau
    stage.react_flow(N, zr, zi, frkc4.react_flow_taus(b, 1.0, nsub), nsub)
    return np.array([zr[0] + 1j * zi[0], zr[1] + 1j * zi[1]])


def _react_ref(tau, y0):
    from scipy.integrate import solve_ivp

    def f(s, y):
        v, w = y[0] + 1j * y[1], y[2] + 1j * y[3]
        fv = tau * (1 - 4 * v + v * v * w)
        fw = tau * (3 * v - v * v * w)
        return [fv.real, fv.imag, fw.real, fw.imag]
    r = solve_ivp(f, (0, 1), [y0[0].real, y0[0].imag, y0[1].real, y0[1].imag], rtol=1e-13,
                  atol=1e-14, method="DOP853").y[:, -1]
    return np.array([r[0] + 1j * r[1], r[2] + 1j * r[3]])


@pytest.mark.parametrize("tau", [0.3, 0.25 + 0.1j, 0.2 - 0.15j])
def test_react_flow_rk4_order(tau):
    """The B flow along a complex time: error against DOP853 falls 16-fold per doubling of
    nsub (classical Runge-Kutta), real and complex tau."""
    y0 = np.array([1.3 + 0.05j, 2.7 - 0.02j])
    ref = _react_ref(tau, y0)
    errs = [np.abs(_react(tau, y0, n) - ref).max() for n in (2, 4, 8)]
    r = errs[0] / errs[1], errs[1] / errs[2]
    assert 13 < r[1] < 19


# ---- the whole scheme ----

def _bruss_rhs(n, h, d=0.02):
    def rhs(t, z):
        v = z[: n * n].reshape(n, n)
        w = z[n * n:].reshape(n, n)
        lap = lambda u: (np.roll(u, 1, 0) + np.roll(u, -1, 0) + np.roll(u, 1, 1)
                         + np.roll(u, -1, 1) - 4 * u) / (h * h)
        return np.concatenate([(d * lap(v) + 1 - 4 * v + w * v * v).ravel(),
                               (d * lap(w) + 3 * v - v * v * w).ravel()])
    return rhs


def test_fourth_order_on_brusselator():
    """Brusselator 32^2 to t = 0.5 with s = 8 and nsub = 4: the error against DOP853 on an
    independent numpy stencil falls about 16-fold per halving of T."""
    from scipy.integrate import solve_ivp
    n = 32
    p = wl.brusselator(n)
    tf = 0.5
    ref = solve_ivp(_bruss_rhs(n, p.h), (0, tf), p.w0.ravel(), rtol=1e-13, atol=1e-13,
                    method="DOP853").y[:, -1]
    rhoA = 8 * p.d_const / p.h ** 2
    c = frkc4.frkc4_coeffs(8, 0.01)
    errs = []
    for m in (4, 8, 16, 32):
        assert tf / m / 4 * rhoA <= c.beta_bar
        errs.append(np.abs(frkc4.run(p, tf / m, 8, m, nsub=4) - ref).max())
    r = [errs[i] / errs[i + 1] for i in range(3)]
    assert 13 < r[-1] < 19 and 11 < r[-2] < 21
