"""Pins of the oracle's error-controlled integration (Sec. 3): the embedded first-order
solution against its closed form on an eigenmode and its order of accuracy, the error norm
against the complex modulus, the stage-count search against a brute-force scan, and the
controller through properties the paper's procedure implies (errors of accepted steps,
the SAFE^2 equilibrium of an O(T^2) estimate, exact arrival at the end time, accuracy that
follows the tolerance on the periodic heat equation, whose Fourier solution is exact)."""
import math

import numpy as np
import pytest

from oracle import adaptive, dense, frkc2_coeffs, stage
from paper_1702_03818_amd import workloads as wl


def mode_problem(N=64, k=3):
    p = wl.Problem(1, (N, 1, 1), 1.0 / N, wl.BC_PERIODIC, wl.OP_LAPLACE, 1.0)
    x = np.arange(N) / N
    p.w0 = np.cos(2 * np.pi * k * x)
    lam = -4.0 * N * N * math.sin(math.pi * k / N) ** 2
    return p, lam


@pytest.mark.parametrize("s", [4, 16, 50])
def test_embedded_solution_closed_form(s):
    """On an eigenvector with eigenvalue lam, W^l = prod_{j<l}(1 + tau_j lam) w and
    What^L = w (1 + sum_l Re(tau_l) lam Re prod_{j<l}(1 + tau_j lam))."""
    p, lam = mode_problem()
    c = frkc2_coeffs(s, 0.01)
    T = 0.5 * c.beta_bar / (4.0 * p.n[0] ** 2)
    tau = T * c.a
    wr, wi, wh = stage.superstep_embedded(p, p.w0, tau.real, tau.imag)
    g = 1.0 + 0j
    acc = 1.0
    for l in range(s):
        acc += tau[l].real * lam * g.real
        g *= 1.0 + tau[l] * lam
    scale = np.max(np.abs(p.w0))
    assert np.max(np.abs(wh - acc * p.w0)) < 1e-12 * scale
    assert np.max(np.abs(wr - g.real * p.w0)) < 1e-12 * scale
    assert np.max(np.abs(wi - g.imag * p.w0)) < 1e-12 * scale


def test_embedded_is_first_order_and_main_second_order():
    """Local error on an eigenmode: What^L - exp(lam T) w = O(T^2), W^L - exp(lam T) w = O(T^3)."""
    p, lam = mode_problem(N=32, k=1)
    c = frkc2_coeffs(16, 0.01)
    errs_h, errs_w = [], []
    for T in (4e-4, 2e-4, 1e-4):
        tau = T * c.a
        wr, wi, wh = stage.superstep_embedded(p, p.w0, tau.real, tau.imag)
        ex = math.exp(lam * T) * p.w0
        errs_h.append(np.max(np.abs(wh - ex)))
        errs_w.append(np.max(np.abs(wr - ex)))
    for a, b in zip(errs_h, errs_h[1:]):
        assert 3.7 < a / b < 4.3
    for a, b in zip(errs_w, errs_w[1:]):
        assert 7.0 < a / b < 9.0


def test_error_norm_is_the_complex_modulus():
    rng = np.random.default_rng(11)
    wr, wi, wh = rng.normal(size=(3, 500))
    tol = 1e-3
    e = adaptive.error_norm(wr, wi, wh, tol)
    ref = max(abs(complex(a, b) - c) / (tol * (1 + max(abs(complex(a, b)), abs(c))))
              for a, b, c in zip(wr, wi, wh))
    assert abs(e - ref) <= 1e-14 * ref
    wr[7] = np.nan
    assert adaptive.error_norm(wr, wi, wh, tol) == math.inf


@pytest.mark.parametrize("x", [1.0, 41.0, 41.7, 168.0, 700.0, 2701.0, 6600.0])
def test_choose_s_is_smallest_covering_s(x):
    s = adaptive.choose_s(x, 0.01)
    assert s % 2 == 0 and 2 <= s <= 514
    assert frkc2_coeffs(s, 0.01).beta_bar >= x
    for q in range(2, s, 2):
        assert frkc2_coeffs(q, 0.01).beta_bar < x


def heat_exact(p, t):
    N = p.n[0]
    x = np.arange(N) / N
    out = np.zeros(N)
    for k, A in zip(p.meta["modes"], p.meta["amplitudes"]):
        lam = -4.0 * N * N * math.sin(math.pi * k / N) ** 2
        out += A * math.exp(lam * t) * np.sin(2 * np.pi * k * x)
    return out


@pytest.mark.parametrize("tol", [1e-3, 1e-5])
def test_controller_properties(tol):
    p = wl.heat1d()
    t_span = 2e-3
    w, trace, T_next = adaptive.integrate(p, t_span, 1e-5, tol)
    acc = [r for r in trace if r[4]]
    rej = [r for r in trace if not r[4]]
    t = 0.0
    for r in acc:
        t = t + r[1]
    assert t == t_span                             # the last step lands on t_span
    assert all(r[3] <= 1.0 for r in acc)
    assert all(r[3] > 1.0 for r in rej)
    rho = stage.rho_bound(p)
    for r in trace:                                # smallest covering stage count
        assert frkc2_coeffs(r[2], 0.01).beta_bar >= r[1] * rho
    # a rejection retries the same start time with T scaled by SAFE / sqrt(err)
    for a, b in zip(trace, trace[1:]):
        if not a[4]:
            assert b[0] == a[0]
            assert b[1] == min(a[1] * (adaptive.SAFE / math.sqrt(a[3])), t_span - a[0])
    # an O(T^2) estimate settles where SAFE/sqrt(err) = 1, i.e. err = SAFE^2
    mid = [r[3] for r in acc[3:-1]]
    assert 0.5 < float(np.median(mid)) < 0.8


def test_accuracy_follows_tolerance():
    p = wl.heat1d()
    t_span = 2e-3
    ex = heat_exact(p, t_span)
    errs, steps = [], []
    for tol in (1e-2, 1e-4, 1e-6):
        w, trace, _ = adaptive.integrate(p, t_span, 1e-5, tol)
        errs.append(np.max(np.abs(w - ex)) / np.max(np.abs(ex)))
        steps.append(len(trace))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 1e-3 and errs[2] < 1e-5
    assert steps[0] < steps[1] < steps[2]


def test_huge_first_step_is_rejected_and_shrunk():
    p = wl.heat1d()
    w, trace, _ = adaptive.integrate(p, 1e-3, 1e-3, 1e-6)
    assert trace[0][4] == 0 and trace[1][1] < trace[0][1]


def test_porous_operator_runs():
    """Nonlinear operator: rho follows the state; the accepted errors stay below 1 and the
    mass of the periodic problem is conserved."""
    p = wl.porous2d(n=64)
    w, trace, _ = adaptive.integrate(p, 2e-4, 1e-6, 1e-4)
    assert all(r[3] <= 1 for r in trace if r[4])
    assert abs(w.sum() - p.w0.sum()) < 1e-10 * abs(p.w0.sum())


def test_user_operator_matches_builtin_operator():
    """Error control around a caller operator (Sec. 3.1 core/user split): the periodic heat
    operator written with numpy takes the same attempts and stage counts as the built-in one
    and ends within rounding of it (the two evaluate the stencil in different orders)."""
    p = wl.heat1d()
    inv_h2 = 1.0 / (p.h * p.h)

    def lap(wr, wi):
        return ((np.roll(wr, 1) + np.roll(wr, -1) - 2.0 * wr) * inv_h2,
                (np.roll(wi, 1) + np.roll(wi, -1) - 2.0 * wi) * inv_h2)

    rho = 4.0 * inv_h2
    w_u, tr_u, _ = adaptive.integrate_user(lap, rho, p.w0, 2000.0 / rho, 100.0 / rho, 1e-4)
    w_b, tr_b, _ = adaptive.integrate(p, 2000.0 / rho, 100.0 / rho, 1e-4)
    assert [(t[2], t[4]) for t in tr_u] == [(t[2], t[4]) for t in tr_b]
    assert np.linalg.norm(w_u - w_b) <= 1e-12 * np.linalg.norm(w_b)


def test_user_scalar_operator_follows_the_stability_polynomial():
    """f = lam W: every accepted step multiplies the state by R(T_n lam) (50-digit product of
    the FP64 stepsizes), so the end state is the product over the accepted steps."""
    lam = -7.0
    w0 = np.linspace(0.5, 1.5, 64)
    w, trace, _ = adaptive.integrate_user(lambda wr, wi: (lam * wr, lam * wi), abs(lam), w0,
                                          3.0, 0.05, 1e-5)
    fac = 1.0
    for t, T, s, err, acc in trace:
        if acc:
            c = adaptive.coeffs(int(s), 0.01)
            fac *= dense.R_hp(c.a, T * lam)
    assert np.max(np.abs(w - fac * w0)) <= 1e-12 * np.max(np.abs(w0))
    assert sum(1 for *_, a in trace if a) > 3


def test_user_rho_function_evaluated_per_accepted_step():
    calls = []

    def rho(w):
        calls.append(float(np.max(np.abs(w))))
        return 3.0

    _, trace, _ = adaptive.integrate_user(lambda wr, wi: (-3.0 * wr, -3.0 * wi), rho,
                                          np.ones(8), 2.0, 0.1, 1e-4)
    accepted = sum(1 for *_, a in trace if a)
    assert len(calls) == accepted   # before the first attempt and after every accept but the last
