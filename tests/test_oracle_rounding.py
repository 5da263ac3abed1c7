"""How far the arithmetic order moves results.

The paper fixes no rounding order. The oracle and the library share one (faces in a fixed
order, each face and the Euler update as correctly rounded fused multiply-adds), which makes
them bit-identical. These tests measure the same supersteps under the plain unfused order (every
multiply-add rounded twice, the oracle built with ORACLE_UNFUSED) at reduced sizes of the
benchmark configurations: the two orders agree far inside the 1e-12 relative L2 gate, so the
gate does not depend on the shared order.
"""
import numpy as np
import pytest

from oracle import frkc2_coeffs, stage
from paper_1702_03818_amd import workloads as wl


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def both(p, w, c, T):
    a = stage.superstep(p, w, T * c.a_re, T * c.a_im)
    b = stage.superstep(p, w, T * c.a_re, T * c.a_im, unfused=True)
    return a, b


def test_orders_differ_at_all():
    """The unfused variant is a different rounding, not the same library twice."""
    p = wl.diffusion3d(n=16, nblobs=2)
    c = frkc2_coeffs(16, 0.01)
    a, b = both(p, p.w0, c, 0.9 * c.beta_bar / stage.rho_bound(p))
    assert not np.array_equal(a, b)


def test_heat1d_full_config():
    """1D heat, N = 1024, s = 16, 20 supersteps (measured 2.7e-15)."""
    p = wl.heat1d()
    c = frkc2_coeffs(16, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p, p.w0)
    a = p.w0.copy()
    b = p.w0.copy()
    for _ in range(20):
        a = stage.superstep(p, a, T * c.a_re, T * c.a_im)
        b = stage.superstep(p, b, T * c.a_re, T * c.a_im, unfused=True)
    assert rel(b, a) < 1e-13


def test_diffusion3d_s100():
    """3D variable D, Dirichlet, 48^3, s = 100, one superstep at T rho = 0.9 betabar
    (measured 1.3-1.4e-14 at 32^3 and 64^3)."""
    p = wl.diffusion3d(n=48)
    c = frkc2_coeffs(100, 0.01)
    a, b = both(p, p.w0, c, 0.9 * c.beta_bar / stage.rho_bound(p))
    assert rel(b, a) < 1e-13


def test_porous2d_s400():
    """2D porous medium, periodic, 256^2, s = 400 at the benchmark's T rho = 0.002 betabar
    (measured 8.6e-15)."""
    p = wl.porous2d(n=256, sigma_cells=4.0)
    c = frkc2_coeffs(400, 0.01)
    a, b = both(p, p.w0, c, 0.002 * c.beta_bar / stage.rho_bound(p, p.w0))
    assert rel(b, a) < 1e-13


def test_adjoint3d_s64():
    """Adjoint configuration at 32^3, s = 64: the forward superstep (measured 3.4e-15) and the
    reverse sweep's lambda (its operator applications use the same fused faces)."""
    p, target = wl.adjoint3d(n=32)
    c = frkc2_coeffs(64, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    a, b = both(p, p.w0, c, T)
    assert rel(b, a) < 1e-13
    lam_a, _ = stage.adjoint(p, p.w0, 2 * (a - target.ravel()), T * c.a_re, T * c.a_im)
    lam_b, _ = stage.adjoint(p, p.w0, 2 * (a - target.ravel()), T * c.a_re, T * c.a_im,
                             unfused=True)
    assert not np.array_equal(lam_a, lam_b)
    assert rel(lam_b, lam_a) < 1e-13
