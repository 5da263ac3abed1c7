"""Pins of the oracle's stage loop, Gershgorin bound and adjoint.

Linear cases are pinned to the exact matrix polynomial R(TA) w (dense brute
force with an independently assembled A, and the Fourier solution of the
periodic heat equation); the nonlinear operator is pinned to an independent
numpy stencil through second-order convergence and mass conservation; the
adjoint is pinned by the dot-product identity and central finite differences.
"""
import numpy as np
import pytest

from oracle import dense, frkc2_coeffs, stage
from paper_1702_03818_amd import workloads as wl


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def test_heat1d_fourier_exact():
    """Periodic 1D heat, N = 1024, s = 16, 20 supersteps: each sine mode k is multiplied by
    R(T lambda_k) per superstep, lambda_k = -4 N^2 sin^2(pi k/N) (exact semi-discrete solution)."""
    p = wl.heat1d()
    N = p.n[0]
    c = frkc2_coeffs(16, 0.01)
    rho = stage.rho_bound(p, p.w0)
    assert rho == 4.0 * N * N
    T = 0.9 * c.beta_bar / rho
    w, _ = stage.run(p, 16, 20, T=T, coeffs=c)
    x = np.arange(N) / N
    exact = np.zeros(N)
    for k, A in zip(p.meta["modes"], p.meta["amplitudes"]):
        lam = -4.0 * N * N * np.sin(np.pi * k / N) ** 2
        exact += A * dense.R_hp(c.a, T * lam) ** 20 * np.sin(2 * np.pi * k * x)
    assert rel(w, exact) < 1e-13


def _tiny(kind):
    if kind == "1d-periodic":
        p = wl.Problem(1, (16, 1, 1), 1.0 / 16, wl.BC_PERIODIC, wl.OP_LAPLACE, 1.0)
    elif kind == "1d-dirichlet-var":
        p = wl.Problem(1, (12, 1, 1), 1.0 / 13, wl.BC_DIRICHLET0, wl.OP_VARCOEF, 1.0,
                       wl.lognormal_D((12,), 2.0, np.random.default_rng(3)))
    elif kind == "2d-dirichlet-var":
        p = wl.Problem(2, (7, 5, 1), 1.0 / 8, wl.BC_DIRICHLET0, wl.OP_VARCOEF, 1.0,
                       wl.lognormal_D((5, 7), 1.5, np.random.default_rng(4)))
    elif kind == "2d-periodic-var":
        p = wl.Problem(2, (6, 8, 1), 1.0 / 8, wl.BC_PERIODIC, wl.OP_VARCOEF, 1.0,
                       wl.lognormal_D((8, 6), 1.5, np.random.default_rng(5)))
    elif kind == "3d-dirichlet-var":
        p = wl.diffusion3d(n=4, nblobs=2)
    elif kind == "3d-periodic-laplace":
        p = wl.Problem(3, (4, 3, 5), 0.25, wl.BC_PERIODIC, wl.OP_LAPLACE, 0.7)
    p.w0 = wl.random_state(p.shape, 11)
    return p


KINDS = ["1d-periodic", "1d-dirichlet-var", "2d-dirichlet-var", "2d-periodic-var",
         "3d-dirichlet-var", "3d-periodic-laplace"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("s", [2, 8, 16, 64, 100])
def test_dense_brute_force(kind, s):
    """Linear superstep equals R(T A) w from eigh of the assembled matrix (Sec. 2)."""
    p = _tiny(kind)
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p, p.w0)
    got = stage.superstep(p, p.w0, T * c.a_re, T * c.a_im)
    ref = dense.superstep(p, p.w0, c.a, T)
    # roundoff grows with the internal amplification Q (Sec. 2.2)
    assert rel(got, ref) < max(1e-14, 1e-15 * c.q_realised) * 10


@pytest.mark.parametrize("kind", KINDS)
def test_rho_bound_is_an_upper_bound(kind):
    """Gershgorin: rho >= the spectral radius of the assembled A (and equal for 1D periodic Laplace)."""
    p = _tiny(kind)
    lam = np.linalg.eigvalsh(dense.assemble(p))
    rho = stage.rho_bound(p, p.w0)
    assert rho >= np.abs(lam).max() * (1 - 1e-12)
    if kind == "1d-periodic":
        assert abs(rho - np.abs(lam).max()) <= 1e-9 * rho


def test_linear_superstep_contracts():
    """|R| <= 1 on the spectrum (T rho <= betabar) and A symmetric: ||w^{n+1}||_2 <= ||w^n||_2."""
    p = wl.diffusion3d(n=12, nblobs=3)
    c = frkc2_coeffs(64, 0.01)
    T = c.beta_bar / stage.rho_bound(p)
    w = p.w0.reshape(-1)
    for _ in range(3):
        w2 = stage.superstep(p, w, T * c.a_re, T * c.a_im)
        assert np.linalg.norm(w2) <= np.linalg.norm(w) * (1 + 1e-14)
        w = w2


def porous_f(u, h):
    """div(u^2 grad u) on a periodic 2D grid, flux form with face value (u_c^2 + u_nb^2)/2, via np.roll."""
    out = np.zeros_like(u)
    for ax in (0, 1):
        for sh in (1, -1):
            un = np.roll(u, sh, axis=ax)
            out += 0.5 * (u * u + un * un) * (un - u)
    return out / (h * h)


def rk4(u, h, t, nsub):
    dt = t / nsub
    for _ in range(nsub):
        k1 = porous_f(u, h)
        k2 = porous_f(u + 0.5 * dt * k1, h)
        k3 = porous_f(u + 0.5 * dt * k2, h)
        k4 = porous_f(u + dt * k3, h)
        u = u + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return u


def test_porous_second_order():
    """Nonlinear u_t = div(u^2 grad u): FRKC2 is second order (Sec. 3), checked against RK4 with
    tiny steps on an independent numpy stencil; error ratio under halving T approaches 4."""
    p = wl.porous2d(n=32, sigma_cells=3.0)
    c = frkc2_coeffs(16, 0.01)
    T0 = 0.9 * c.beta_bar / stage.rho_bound(p, p.w0)
    tf = T0
    ref = rk4(p.w0.copy(), p.h, tf, 8000)
    errs = []
    for m in (16, 32, 64, 128):
        w, _ = stage.run(p, 16, m, T=tf / m, coeffs=c)
        errs.append(np.linalg.norm(w.reshape(p.shape) - ref))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    # pre-asymptotic at the largest T; the ratios fall monotonically towards 2^2
    assert ratios[0] > ratios[1] > ratios[2]
    assert 3.8 < ratios[2] < 4.2


def test_porous_operator_matches_numpy_stencil():
    """One two-stage superstep with s = 2 (RK2): compare with RK2 written on the numpy stencil."""
    p = wl.porous2d(n=16, sigma_cells=2.0)
    c = frkc2_coeffs(2, 0.0)
    T = 1e-4
    got = stage.superstep(p, p.w0, T * c.a_re, T * c.a_im)
    u = p.w0
    k1 = porous_f(u, p.h)
    # a = (1 +- i)/2: W1 = u + T a1 f(u), W2 = W1 + T a2 f(W1), real result = RK2 midpoint-free form
    a1, a2 = complex(c.a_re[0], c.a_im[0]), complex(c.a_re[1], c.a_im[1])
    w1 = u + T * a1 * k1
    fw1 = porous_f_complex(w1, p.h)
    ref = (w1 + T * a2 * fw1).real
    assert rel(got, ref) < 1e-14


def porous_f_complex(u, h):
    out = np.zeros_like(u, dtype=np.complex128)
    for ax in (0, 1):
        for sh in (1, -1):
            un = np.roll(u, sh, axis=ax)
            out += 0.5 * (u * u + un * un) * (un - u)
    return out / (h * h)


def test_periodic_mass_conservation():
    """Flux form on a periodic grid: sum of w is conserved by every stage (to roundoff)."""
    p = wl.porous2d(n=64, sigma_cells=4.0)
    c = frkc2_coeffs(16, 0.01)
    w, _ = stage.run(p, 16, 3, cfl=0.5, coeffs=c)
    assert np.isfinite(w).all()
    assert abs(w.sum() - p.w0.sum()) <= 1e-13 * abs(p.w0.sum())


def test_porous_complex_stages_limit_T():
    """Characterisation (not a pin): with u-dependent diffusivity the complex stages make the
    face value W^2 complex, which turns the high-frequency spectrum off the real axis where the
    stability domain is thin. At s = 100 the superstep stays bounded for T rho = 0.03 betabar
    but diverges at T rho = 0.9 betabar."""
    p = wl.porous2d(n=128, sigma_cells=4.0)
    c = frkc2_coeffs(100, 0.01)
    w, _ = stage.run(p, 100, 3, cfl=0.03, coeffs=c)
    assert np.isfinite(w).all() and np.abs(w).max() < 1.6
    with np.errstate(all="ignore"):
        try:
            w, _ = stage.run(p, 100, 3, cfl=0.9, coeffs=c)
            diverged = not (np.isfinite(w).all() and np.abs(w).max() < 1.6)
        except ZeroDivisionError:
            diverged = True
    assert diverged


def _max_stable_cfl(p, s, steps=3, iters=10):
    """Largest cfl (bisection on [0, 1]) for which `steps` supersteps stay bounded."""
    c = frkc2_coeffs(s, 0.01)

    def ok(cfl):
        with np.errstate(all="ignore"):
            try:
                w, _ = stage.run(p, s, steps, cfl=cfl, coeffs=c)
            except ZeroDivisionError:
                return False
        return bool(np.isfinite(w).all() and np.abs(w).max() < 1.6)

    if ok(1.0):
        return 1.0, c
    lo, hi = 0.0, 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if ok(mid) else (lo, mid)
    return lo, c


def test_porous_stable_step_saturates_in_s():
    """Characterisation (not a pin) of the porous operator with complex stages: small s run
    at the full T rho = betabar(s); from s ~ 64 on the longest stable step no longer grows
    with s (T rho ~ 500 on 32^2, ~1000 on 64^2 and 128^2), so larger s buy no longer steps."""
    p = wl.porous2d(n=32, sigma_cells=4.0)
    cfl16, _ = _max_stable_cfl(p, 16)
    assert cfl16 == 1.0
    cfl64, c64 = _max_stable_cfl(p, 64)
    cfl100, c100 = _max_stable_cfl(p, 100)
    t64, t100 = cfl64 * c64.beta_bar, cfl100 * c100.beta_bar
    assert 300 < t64 and t100 < 1.5 * t64 and cfl100 < 0.2


def test_superstep_linearity():
    """Linear f: S(alpha u + v) = alpha S(u) + S(v)."""
    p = wl.diffusion3d(n=10, nblobs=2)
    c = frkc2_coeffs(100, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    u = wl.random_state(p.shape, 1, smooth=1.5).reshape(-1)
    v = wl.random_state(p.shape, 2, smooth=1.5).reshape(-1)
    lhs = stage.superstep(p, 2.5 * u + v, T * c.a_re, T * c.a_im)
    rhs = 2.5 * stage.superstep(p, u, T * c.a_re, T * c.a_im) + stage.superstep(p, v, T * c.a_re, T * c.a_im)
    assert rel(lhs, rhs) < 1e-12


def _adj_problem(kind):
    if kind == "3d":
        p = wl.diffusion3d(n=6, nblobs=2, n_xyz=(6, 5, 4))
    else:
        p = _tiny("2d-periodic-var")
    p.w0 = wl.random_state(p.shape, 21, smooth=1.0).reshape(-1)
    return p


@pytest.mark.parametrize("kind", ["3d", "2d-periodic"])
def test_adjoint_dot_product(kind):
    """<S u, v> = <u, S^T v>: the reverse stage sequence with conj(tau) is the transpose."""
    p = _adj_problem(kind)
    c = frkc2_coeffs(16, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    tr, ti = T * c.a_re, T * c.a_im
    v = wl.random_state(p.shape, 22).reshape(-1)
    Su = stage.superstep(p, p.w0, tr, ti)
    lam, _ = stage.adjoint(p, p.w0, v, tr, ti)
    assert abs(Su @ v - p.w0 @ lam) <= 1e-13 * np.linalg.norm(Su) * np.linalg.norm(v)


@pytest.mark.parametrize("kind", ["3d", "2d-periodic"])
def test_adjoint_logD_central_differences(kind):
    """dJ/dlogD of J = <S_D(w), v> against central differences (step 1e-5) in seeded directions."""
    p = _adj_problem(kind)
    c = frkc2_coeffs(16, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    tr, ti = T * c.a_re, T * c.a_im
    v = wl.random_state(p.shape, 23).reshape(-1)
    logD = np.log(p.D.reshape(-1))
    _, g = stage.adjoint(p, p.w0, v, tr, ti)
    rng = np.random.default_rng(24)
    eps = 1e-5
    for _ in range(4):
        d = rng.standard_normal(logD.shape)
        jp = stage.superstep(p, p.w0, tr, ti, D=np.exp(logD + eps * d)) @ v
        jm = stage.superstep(p, p.w0, tr, ti, D=np.exp(logD - eps * d)) @ v
        fd = (jp - jm) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-7 * max(1.0, abs(fd))


def test_adjoint_chain_two_supersteps():
    """Quadratic loss over two supersteps: gradient in w0 against central differences (exact
    for a quadratic) and the logD gradient accumulated over both supersteps."""
    p = _adj_problem("3d")
    c = frkc2_coeffs(8, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    tr, ti = T * c.a_re, T * c.a_im
    target = wl.random_state(p.shape, 25).reshape(-1)

    def J(w0, D):
        w1 = stage.superstep(p, w0, tr, ti, D=D)
        w2 = stage.superstep(p, w1, tr, ti, D=D)
        return float(((w2 - target) ** 2).sum()), w1, w2

    j0, w1, w2 = J(p.w0, p.D)
    lam2 = 2 * (w2 - target)
    g = np.zeros(p.npoints)
    lam1, g = stage.adjoint(p, w1, lam2, tr, ti, grad_logD=g)
    lam0, g = stage.adjoint(p, p.w0, lam1, tr, ti, grad_logD=g)
    rng = np.random.default_rng(26)
    for _ in range(3):
        d = rng.standard_normal(p.npoints)
        fd = (J(p.w0 + 1e-3 * d, p.D)[0] - J(p.w0 - 1e-3 * d, p.D)[0]) / 2e-3
        assert abs(fd - lam0 @ d) <= 1e-9 * max(1.0, abs(fd))
        logD = np.log(p.D.reshape(-1))
        fd = (J(p.w0, np.exp(logD + 1e-5 * d))[0] - J(p.w0, np.exp(logD - 1e-5 * d))[0]) / 2e-5
        assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd))


def test_face_mean_halves_are_the_plain_mean():
    """The face rules take D_c/2 + D_nb/2 (and W_c^2/2 + W_nb^2/2 with the imaginary half formed
    as re*im): scaling by 2 commutes with rounding, so for normal values these are the plain
    means (a + b)/2 bit for bit. Checked on random pairs over a wide exponent range, both
    signs, including pairs that cancel."""
    rng = np.random.default_rng(7)
    n = 1_000_000
    a = np.exp(rng.uniform(-300, 300, n)) * rng.choice([-1.0, 1.0], n)
    b = np.where(rng.random(n) < 0.1, -a * (1 + 1e-12 * rng.standard_normal(n)),
                 np.exp(rng.uniform(-300, 300, n)) * rng.choice([-1.0, 1.0], n))
    assert np.array_equal(0.5 * a + 0.5 * b, 0.5 * (a + b))
    x = rng.standard_normal(n) * np.exp(rng.uniform(-100, 100, n))
    y = rng.standard_normal(n) * np.exp(rng.uniform(-100, 100, n))
    assert np.array_equal(x * y, 0.5 * (2.0 * (x * y)))
