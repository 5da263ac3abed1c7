"""Pins of the oracle's nonlinear operator div(u^2 grad u) off the 2D periodic grid and of its
Gershgorin bound (Sec. 2: the stability requirement T rho <= betabar needs rho to bound the
spectral radius of the Jacobian of f, here state dependent).

The reference operator below is written independently of the oracle: numpy array shifts with a
zero ghost layer for Dirichlet boundaries (np.roll for periodic ones), in the flux form with
face value (u_c^2 + u_nb^2)/2, in complex arithmetic so it applies to the complex stage values.
"""
import numpy as np
import pytest

from oracle import frkc2_coeffs, stage
from paper_1702_03818_amd import workloads as wl


def shift(u, ax, sh, periodic):
    """u at the neighbour sh (+1 or -1) cells along axis ax; zero outside a Dirichlet grid."""
    if periodic:
        return np.roll(u, -sh, axis=ax)
    out = np.zeros_like(u)
    src = [slice(None)] * u.ndim
    dst = [slice(None)] * u.ndim
    if sh > 0:
        src[ax], dst[ax] = slice(1, None), slice(0, -1)
    else:
        src[ax], dst[ax] = slice(0, -1), slice(1, None)
    out[tuple(dst)] = u[tuple(src)]
    return out


def porous_f(u, h, periodic):
    out = np.zeros_like(u)
    for ax in range(u.ndim):
        for sh in (-1, 1):
            un = shift(u, ax, sh, periodic)
            out = out + 0.5 * (u * u + un * un) * (un - u)
    return out / (h * h)


def problem(ndim, bc, n, seed, rough):
    shape = {1: (n,), 2: (n + 1, n), 3: (n - 1, n + 1, n)}[ndim]
    nn = tuple(reversed(shape)) + (1,) * (3 - ndim)
    h = 1.0 / (n + 1) if bc == wl.BC_DIRICHLET0 else 1.0 / n
    p = wl.Problem(ndim, nn, h, bc, wl.OP_POROUS2, 1.0)
    g = wl.random_state(shape, seed, smooth=None if rough else 1.5)
    p.w0 = np.ascontiguousarray(1.0 + (0.8 if rough else 0.45) * g / np.abs(g).max())
    return p


CASES = [(d, bc) for d in (1, 2, 3) for bc in (wl.BC_PERIODIC, wl.BC_DIRICHLET0)]


@pytest.mark.parametrize("ndim,bc", CASES)
@pytest.mark.parametrize("rough", [False, True])
def test_rho_bounds_the_fd_jacobian(ndim, bc, rough):
    """rho >= max |eigenvalue| of the finite-difference Jacobian of the reference operator at
    seeded smooth and rough states, and within a factor 1.5 of it (a Gershgorin row sum, not a
    loose constant)."""
    n = {1: 24, 2: 7, 3: 4}[ndim]
    p = problem(ndim, bc, n, 31 + ndim, rough)
    per = bc == wl.BC_PERIODIC
    x = p.w0.astype(float)
    N = x.size
    J = np.zeros((N, N))
    eps = 1e-6
    for j in range(N):
        e = np.zeros(N)
        e[j] = eps
        J[:, j] = (porous_f((x.ravel() + e).reshape(x.shape), p.h, per)
                   - porous_f((x.ravel() - e).reshape(x.shape), p.h, per)).ravel() / (2 * eps)
    lam = np.max(np.abs(np.linalg.eigvals(J)))
    rho = stage.rho_bound(p, x)
    assert lam <= rho * (1 + 1e-7)
    assert rho <= 1.5 * lam


def test_rho_exact_on_alternating_state():
    """1D periodic, w alternating 1.5 / 0.5: every row has |diag| + sum|off| = 7/h^2, and the
    Jacobian's spectral radius is exactly that (the alternating mode); the frozen-coefficient
    value (2/h^2) sum_f Q_f = 5/h^2 would not bound it."""
    n = 64
    p = wl.Problem(1, (n, 1, 1), 1.0 / n, wl.BC_PERIODIC, wl.OP_POROUS2, 1.0)
    w = np.where(np.arange(n) % 2 == 0, 1.5, 0.5)
    assert stage.rho_bound(p, w) == 7.0 * n * n


@pytest.mark.parametrize("ndim,bc", CASES)
def test_rk2_identity(ndim, bc):
    """s = 2 gives a = (1 +- i)/2: the superstep equals the two complex Euler steps written on
    the reference operator (Dirichlet ghosts and the 1D and 3D forms included)."""
    n = {1: 40, 2: 12, 3: 6}[ndim]
    p = problem(ndim, bc, n, 41 + ndim, rough=False)
    per = bc == wl.BC_PERIODIC
    c = frkc2_coeffs(2, 0.0)
    T = 0.5 / stage.rho_bound(p, p.w0)
    got = stage.superstep(p, p.w0, T * c.a_re, T * c.a_im)
    a1, a2 = complex(c.a_re[0], c.a_im[0]), complex(c.a_re[1], c.a_im[1])
    u = p.w0.astype(complex)
    w1 = u + T * a1 * porous_f(u, p.h, per)
    ref = (w1 + T * a2 * porous_f(w1, p.h, per)).real
    assert np.linalg.norm(got.ravel() - ref.ravel()) <= 1e-14 * np.linalg.norm(ref)


@pytest.mark.parametrize("ndim", [1, 3])
def test_second_order_dirichlet(ndim):
    """Dirichlet-zero grids in 1D and 3D: error ratio under halving T approaches 4 against RK4
    with small steps on the reference operator."""
    n = {1: 48, 3: 6}[ndim]
    p = problem(ndim, wl.BC_DIRICHLET0, n, 51 + ndim, rough=False)
    c = frkc2_coeffs(8, 0.01)
    tf = 0.9 * c.beta_bar / stage.rho_bound(p, p.w0)
    u = p.w0.copy()
    nsub = 4000
    dt = tf / nsub
    for _ in range(nsub):
        k1 = porous_f(u, p.h, False)
        k2 = porous_f(u + 0.5 * dt * k1, p.h, False)
        k3 = porous_f(u + 0.5 * dt * k2, p.h, False)
        k4 = porous_f(u + dt * k3, p.h, False)
        u = u + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    errs = []
    for m in (8, 16, 32, 64):
        w, _ = stage.run(p, 8, m, T=tf / m, coeffs=c)
        errs.append(np.linalg.norm(w.reshape(p.w0.shape) - u))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert 3.7 < ratios[-1] < 4.3
