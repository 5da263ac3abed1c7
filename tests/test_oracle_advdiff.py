"""Pins of the oracle's advection-diffusion operator (central differences) and of damping
(Sec. 2.1: damping widens the stability domain off the real axis so that problems with a small
hyperbolic part can be run): Fourier eigenmodes against the stability polynomial, the Gershgorin
bound against the eigenvalues of an independently assembled matrix, and growth without damping
against decay with it."""
import math

import numpy as np
import pytest

from oracle import dense, frkc2_coeffs, stage
from paper_1702_03818_amd import workloads as wl


def adv_problem(n, vel, d=1.0, bc=wl.BC_PERIODIC):
    ndim = len(n)
    nn = tuple(n) + (1,) * (3 - ndim)
    p = wl.Problem(ndim, nn, 1.0 / n[0], bc, wl.OP_ADVDIFF, d)
    p.vel = tuple(vel) + (0.0,) * (3 - len(vel))
    return p


def mode_lambda(p, thetas):
    """Eigenvalue of the central advection-diffusion stencil for phases theta per cell."""
    lam = 0.0
    for k, th in enumerate(thetas):
        fm = p.d_const + 0.5 * p.h * p.vel[k]
        fp = p.d_const - 0.5 * p.h * p.vel[k]
        lam += fm * (np.exp(-1j * th) - 1) + fp * (np.exp(1j * th) - 1)
    return lam / (p.h * p.h)


@pytest.mark.parametrize("n,vel,kk", [((64,), (10.0,), (3,)), ((32, 24), (6.0, -4.0), (2, 5))])
def test_fourier_mode(n, vel, kk):
    p = adv_problem(n, vel)
    c = frkc2_coeffs(16, 0.1)
    rho = stage.rho_bound(p)
    T = 0.9 * c.beta_bar / rho
    grids = np.meshgrid(*[np.arange(m) for m in n[::-1]], indexing="ij")[::-1]
    thetas = [2 * math.pi * k / m for k, m in zip(kk, n)]
    phase = sum(th * g for th, g in zip(thetas, grids))
    w0 = np.cos(phase)
    out = stage.superstep(p, w0, T * c.a_re, T * c.a_im)
    R = dense.R_hp_complex(c.a, T * mode_lambda(p, thetas))
    ref = (R * np.exp(1j * phase)).real
    assert np.max(np.abs(out.reshape(ref.shape) - ref)) < 1e-12


def test_gershgorin_bounds_the_spectrum():
    p = adv_problem((24,), (30.0,), bc=wl.BC_DIRICHLET0)
    n = 24
    fm = p.d_const + 0.5 * p.h * p.vel[0]
    fp = p.d_const - 0.5 * p.h * p.vel[0]
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] = -(fm + fp)
        if i > 0:
            A[i, i - 1] = fm
        if i + 1 < n:
            A[i, i + 1] = fp
    A /= p.h * p.h
    lam = np.max(np.abs(np.linalg.eigvals(A)))
    assert lam <= stage.rho_bound(p) and lam > 0.5 * stage.rho_bound(p)


def test_damping_stabilises_a_small_hyperbolic_part():
    """Peclet number v L / d = 10 on the periodic unit line, s = 16, T rho = betabar: without
    damping a mode has |R| > 1 and the state grows; with nu = 0.1 every |R| <= 1 and it does not
    (the extent betabar shrinks by about nu, Sec. 2.1)."""
    N = 64
    p = adv_problem((N,), (10.0,))
    rng = np.random.default_rng(1)
    w0 = rng.standard_normal(N)
    norms = {}
    for nu in (0.0, 0.1):
        c = frkc2_coeffs(16, nu)
        T = c.beta_bar / stage.rho_bound(p)
        ths = 2 * math.pi * np.arange(N) / N
        rmax = max(abs(dense.R_hp_complex(c.a, T * mode_lambda(p, [t]))) for t in ths)
        w = w0.copy()
        for _ in range(40):
            w = stage.superstep(p, w, T * c.a_re, T * c.a_im)
        norms[nu] = (rmax, np.linalg.norm(w) / np.linalg.norm(w0))
    assert norms[0.0][0] > 1.05 and norms[0.0][1] > 5.0
    assert norms[0.1][0] <= 1.0 + 1e-12 and norms[0.1][1] <= 1.0
