"""Pins of the damping sweep (Sec. 2.1, "Damping"): the smallest nu for which every Fourier mode
of a periodic advection-diffusion problem is stable at T = betabar(nu)/rho.

Independent checks: the Fourier symbols against the eigenvalues of a matrix assembled here with
np.roll; the Gershgorin bound against the stage oracle's; the extent shrinking by about (1 - nu)
(the paper's statement); minimality of the nu found, with R evaluated in 50-digit arithmetic;
and the dynamics: supersteps of the stage oracle grow at the next smaller nu and decay at the
one found. The table of nu against the Peclet number that the design notes quote is checked last.
"""
import numpy as np
import pytest

from oracle import damping, dense, frkc2_coeffs, stage
from paper_1702_03818_amd import workloads as wl


def problem(n, vel, d=1.0):
    ndim = len(n)
    p = wl.Problem(ndim, tuple(n) + (1,) * (3 - ndim), 1.0 / n[0], wl.BC_PERIODIC,
                   wl.OP_ADVDIFF, d)
    p.vel = tuple(vel) + (0.0,) * (3 - ndim)
    return p


def assembled(n, h, d, vel):
    """Matrix of the periodic central stencil, built cell by cell with np.roll (x fastest)."""
    shape = tuple(reversed(n))
    N = int(np.prod(n))
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        u = e.reshape(shape)
        out = np.zeros(shape)
        for k, v in enumerate(vel):
            ax = len(n) - 1 - k
            cm, cp = d + 0.5 * h * v, d - 0.5 * h * v
            out += cm * (np.roll(u, 1, axis=ax) - u) + cp * (np.roll(u, -1, axis=ax) - u)
        A[:, j] = out.reshape(-1) / (h * h)
    return A


@pytest.mark.parametrize("n,vel", [((12,), (30.0,)), ((6, 5), (7.0, -3.0)), ((4, 3, 5), (2.0, 9.0, -6.0))])
def test_symbols_are_the_eigenvalues(n, vel):
    h, d = 1.0 / n[0], 0.7
    lam = damping.symbols(n, h, d, vel)
    ev = np.linalg.eigvals(assembled(n, h, d, vel))
    assert lam.size == ev.size
    # every assembled eigenvalue has a symbol within rounding, and the other way round
    scale = np.abs(ev).max()
    for a, b in ((ev, lam), (lam, ev)):
        dist = np.abs(a[:, None] - b[None, :]).min(axis=1)
        assert dist.max() <= 1e-9 * scale


@pytest.mark.parametrize("vel,d", [((10.0,), 1.0), ((300.0,), 1.0), ((6.0, -4.0), 0.5),
                                   ((1.0, 2.0, -3.0), 2.0)])
def test_gershgorin_is_the_stage_oracles(vel, d):
    n = (32,) * len(vel)
    p = problem(n, vel, d)
    assert damping.gershgorin(p.h, d, vel) == stage.rho_bound(p)


@pytest.mark.parametrize("nu", [0.02, 0.08, 0.25])
@pytest.mark.parametrize("s", [16, 50, 100])
def test_extent_shrinks_by_about_one_minus_nu(nu, s):
    """Sec. 2.1: damping costs about a factor (1 - nu) of the real extent."""
    r = frkc2_coeffs(s, nu).beta / frkc2_coeffs(s, 0.0).beta
    assert abs(r / (1.0 - nu) - 1.0) < 0.01


@pytest.mark.parametrize("n,vel,s", [((64,), (10.0,), 16), ((32, 24), (6.0, -4.0), 16),
                                     ((256,), (20.0,), 50)])
def test_found_damping_is_the_smallest(n, vel, s):
    """At the nu found every mode has |R| <= 1; at the grid value below it some mode has
    |R| > 1 (both decided on the worst modes in 50-digit arithmetic)."""
    h, d = 1.0 / n[0], 1.0
    r = damping.min_damping(n, h, d, vel, s)
    assert r is not None and r["nu"] > 0
    lam = damping.symbols(n, h, d, vel)
    rho = damping.gershgorin(h, d, vel)
    for nu, stable in ((r["nu"], True), (round(r["nu"] - 0.01, 10), False)):
        c = frkc2_coeffs(s, nu)
        T = c.beta_bar / rho
        la = damping.log_amplification(c.a, T * lam)
        worst = [abs(dense.R_hp_complex(c.a, T * lam[i])) for i in np.argsort(la)[-4:]]
        if stable:
            assert max(worst) <= 1.0 + 1e-12
        else:
            assert max(worst) > 1.0 + 1e-6


def test_supersteps_grow_below_and_decay_at_the_found_damping():
    """Peclet 10 on 64 periodic cells, s = 16: 400 supersteps of the stage oracle from a random
    state grow by orders of magnitude at nu - 0.01 and do not grow at nu."""
    n, vel, s = (64,), (10.0,), 16
    p = problem(n, vel)
    r = damping.min_damping(n, p.h, 1.0, vel, s)
    rho = stage.rho_bound(p)
    w0 = np.random.default_rng(1).standard_normal(64)
    growth = {}
    for nu in (round(r["nu"] - 0.01, 10), r["nu"]):
        c = frkc2_coeffs(s, nu)
        T = c.beta_bar / rho
        w = w0.copy()
        for _ in range(400):
            w = stage.superstep(p, w, T * c.a_re, T * c.a_im)
        growth[nu] = np.linalg.norm(w) / np.linalg.norm(w0)
    lo, hi = sorted(growth)
    assert growth[lo] > 1e3 and growth[hi] <= 1.0


# nu found per Peclet number v L / d (L the period): 64 cells with s = 16, 256 cells with s = 50
TABLE = {(64, 16): {1: 0.01, 5: 0.03, 10: 0.08, 20: 0.26},
         (256, 50): {1: 0.01, 5: 0.02, 10: 0.05, 20: 0.18}}


@pytest.mark.parametrize("N,s", sorted(TABLE))
def test_damping_per_peclet_number(N, s):
    """The sweep's table: more damping for larger Peclet numbers, and the real extent lost is
    within 5 % of nu (the figures the design notes quote)."""
    prev = 0.0
    for pe, nu in sorted(TABLE[(N, s)].items()):
        r = damping.min_damping((N,), 1.0 / N, 1.0, (float(pe),), s)
        assert r["nu"] == nu and r["nu"] >= prev
        assert abs((1.0 - r["beta"] / r["beta0"]) / nu - 1.0) < 0.05
        prev = r["nu"]
