"""Pins of the oracle's stepsizes against what the paper and the mathematics fix.

Each test names the property it pins and where it comes from. None of them
re-types the oracle's own formula: they check order conditions, a textbook
special case, a closed form derived independently through the Chebyshev
expansion, printed numbers of the paper, and brute-force scans.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import coeffs as oc
from oracle.coeffs import frkc2_coeffs


def elem_sym(a, k):
    """Elementary symmetric polynomial e_k of the stepsizes, via Newton's identities in mpmath.

    R(x) = prod (1 + a_l x) = sum_k e_k x^k, so R^{(k)}(0) = k! e_k.
    """
    with mp.workdps(60):
        av = [mp.mpc(float(v.real), float(v.imag)) for v in a]
        p = [None] + [mp.fsum([v ** j for v in av]) for j in range(1, k + 1)]
        e = [mp.mpc(1)]
        for j in range(1, k + 1):
            e.append(mp.fsum([(-1) ** (i - 1) * e[j - i] * p[i] for i in range(1, j + 1)]) / j)
        return e[k]


@pytest.mark.parametrize("nu", [0.0, 0.01, 0.2])
def test_two_stages_is_rk2(nu):
    """L = 2: the only second-order two-stage Euler product is R = 1 + x + x^2/2 (textbook RK2)."""
    c = frkc2_coeffs(2, nu)
    a = np.sort_complex(c.a)
    assert np.allclose(a, [0.5 - 0.5j, 0.5 + 0.5j], rtol=0, atol=1e-15)
    poly = np.polynomial.polynomial.polyfromroots(-1.0 / c.a)
    poly = poly / poly[0]
    assert np.allclose(poly, [1.0, 1.0, 0.5], atol=1e-15)
    assert c.beta == 2.0  # RK2 real-axis stability limit


@pytest.mark.parametrize("s", [4, 8, 16, 64, 100, 200, 400])
@pytest.mark.parametrize("nu", [0.0, 0.01])
def test_order_conditions(s, nu):
    """Linear order conditions R'(0) = R''(0) = 1 (Sec. 2, eq. 'order')."""
    c = frkc2_coeffs(s, nu)
    e1 = elem_sym(c.a, 1)
    e2 = elem_sym(c.a, 2)
    assert abs(e1 - 1) < 1e-14 * s
    assert abs(2 * e2 - 1) < 1e-13 * s


@pytest.mark.parametrize("s", [4, 8, 16, 64, 100, 400])
def test_undamped_third_derivative(s):
    """nu = 0: R'''(0) = 0.6 (L^2 - 4)/(L^2 - 1), from the Chebyshev form c0 + C_L(1 + 3x/(L^2-1))."""
    c = frkc2_coeffs(s, 0.0)
    L = s
    r3 = 6 * elem_sym(c.a, 3)
    assert abs(r3 - 0.6 * (L * L - 4) / (L * L - 1)) < 1e-12


@pytest.mark.parametrize("s", [4, 16, 100])
def test_undamped_closed_form(s):
    """nu = 0: the product of Euler factors equals (2L^2+1)/(3L^2) + (L^2-1)/(3L^2) T_L(1 + 3x/(L^2-1)).

    The right side is written with numpy's Chebyshev class (an independent
    evaluation of T_L); the left side is the product in 50-digit arithmetic of
    the FP64 stepsizes.
    """
    c = frkc2_coeffs(s, 0.0)
    L = s
    TL = np.polynomial.chebyshev.Chebyshev.basis(L)
    xs = np.linspace(-2 * (L * L - 1) / 3, 0, 57)
    for x in xs:
        with mp.workdps(50):
            r = mp.mpc(1)
            for al in c.a:
                r *= 1 + mp.mpc(float(al.real), float(al.imag)) * x
        closed = (2 * L * L + 1) / (3 * L * L) + (L * L - 1) / (3 * L * L) * TL(1 + 3 * x / (L * L - 1))
        assert abs(float(mp.re(r)) - closed) < 1e-12
        assert abs(float(mp.im(r))) < 1e-12


def test_undamped_mu_is_zero():
    """nu = 0 leaves the closed-form roots untouched: mu = 0 solves the order conditions."""
    _, mu, _ = oc.damped_group(16, 0.0)
    assert abs(mu) < 1e-40


@pytest.mark.parametrize("s", [4, 16, 100, 400])
def test_undamped_extent(s):
    """nu = 0: beta = 2 M^2 alpha_M = 2 (L^2 - 1)/3 (end point where C_L(z) = 1 at z = -1)."""
    c = frkc2_coeffs(s, 0.0)
    beta0 = 2 * (s * s - 1) / 3
    assert abs(c.beta - beta0) <= 1e-12 * beta0


def test_extent_ratio_printed(paper_numbers):
    """beta / (L^2 beta_RK2) = 0.330 for FRKC2 (Sec. 2, Fig. 1); damping nu = 0.01."""
    ref = paper_numbers["extent_ratio_frkc2"]["value"]
    for s in (100, 200, 400):
        c = frkc2_coeffs(s, 0.01)
        assert round(c.beta / (2.0 * s * s), 3) == ref


@pytest.mark.parametrize("nu", [0.01, 0.05, 0.1])
def test_damping_shrinks_extent_by_one_minus_nu(nu):
    """Sec. 2.1: damping reduces beta by approximately (1 - nu)."""
    s = 100
    c = frkc2_coeffs(s, nu)
    beta0 = 2 * (s * s - 1) / 3
    assert abs(c.beta / beta0 - (1 - nu)) < 0.1 * nu


@pytest.mark.parametrize("s", [16, 100])
def test_damping_lowers_interior_maxima(s):
    """Sec. 2.1: the marginal maxima |R| = 1 inside the interval drop to about 1 - nu0 (nu0 = 2 nu).

    Brute-force scan of |R| on [-0.9 beta, -beta/10] for nu = 0 (maxima at 1)
    and nu = 0.01 (maxima below 1, near 0.97-0.98).
    """
    for nu, lo, hi in [(0.0, 1 - 1e-9, 1 + 1e-9), (0.01, 0.95, 0.99)]:
        c = frkc2_coeffs(s, nu)
        x = np.linspace(-0.9 * c.beta, -0.1 * c.beta, 20001)
        r = np.exp(2 * oc.log_abs_R_half(c.a_re[: s // 2], c.a_im[: s // 2], x))
        assert lo <= r.max() <= hi


@pytest.mark.parametrize("s", [4, 8, 16, 64, 100, 200, 400])
def test_extent_is_stable_and_tight(s):
    """|R| <= 1 on a brute-force grid of [-beta, 0] and |R| > 1 just beyond -beta."""
    c = frkc2_coeffs(s, 0.01)
    x = np.linspace(-c.beta, 0.0, 200001)
    half = slice(0, s // 2)
    lr = 2 * oc.log_abs_R_half(c.a_re[half], c.a_im[half], x)
    assert lr.max() <= 1e-12
    beyond = 2 * oc.log_abs_R_half(c.a_re[half], c.a_im[half], [-c.beta * (1 + 1e-6)])
    assert beyond[0] > 0


@pytest.mark.parametrize("s", [4, 16, 100, 400])
def test_conjugate_halves(s):
    """Second half of the stage sequence is the exact conjugate of the first (real polynomial)."""
    c = frkc2_coeffs(s, 0.01)
    M = s // 2
    assert np.array_equal(c.a_re[M:], c.a_re[:M])
    assert np.array_equal(c.a_im[M:], -c.a_im[:M])


def test_ordering_bound_for_config_stage_counts(paper_numbers):
    """Sec. 2.2: realised Q <= 10 L^2 and at least about L^2/3 (optimum is about L^2).

    Q is re-measured here by brute force over all runs (j, k), independently of
    the oracle's Kadane scan.
    """
    fac = paper_numbers["q_practical_bound_factor"]["value"]
    for s in (8, 16, 64, 100, 200, 400):
        c = frkc2_coeffs(s, 0.01)
        assert c.q_bound_met and c.q_realised <= fac * s * s
        x = np.linspace(-c.beta, 0.0, 1500)
        lf = np.log(np.abs(1.0 + np.outer(c.a, x)))  # s x G
        cs = np.vstack([np.zeros(len(x)), np.cumsum(lf, axis=0)])
        best = -np.inf
        for j in range(s):
            best = max(best, (cs[j + 1:] - cs[j]).max())
        q_brute = math.exp(best)
        assert q_brute <= c.q_realised * (1 + 1e-9)
        assert q_brute >= 0.3 * s * s


def test_ordering_is_essential():
    """Natural root order (each root followed by its conjugate) drowns FP64: Q far above 10 L^2."""
    s = 100
    c = frkc2_coeffs(s, 0.01)
    a_g, _, _ = oc.damped_group(s, 0.01)   # first group in root-index order
    nat = np.array([complex(v) for v in a_g])
    seq = np.ravel(np.column_stack([nat, np.conj(nat)]))
    assert oc.realised_q(seq, c.beta, s) > 1e6 * s * s


def test_reversed_sequence_same_q():
    """Contiguous runs of the reversed sequence are the runs of the original: Q is reversal invariant.

    (This is why the adjoint, which runs the stages backwards, is as stable.)
    """
    c = frkc2_coeffs(64, 0.01)
    q1 = oc.realised_q(c.a, c.beta, 64)
    q2 = oc.realised_q(c.a[::-1], c.beta, 64)
    assert abs(q1 - q2) <= 1e-12 * q1


@pytest.mark.slow
def test_mean_shrink_count(paper_numbers):
    """Sec. 2.2: mean n over the second-order schemes is about 1.5; Q <= 10 L^2 for every even L <= 200."""
    ns = []
    for s in range(8, 201, 2):
        c = frkc2_coeffs(s, 0.01)
        assert c.q_bound_met, s
        ns.append(c.n_shrink)
    mean_n = float(np.mean(ns))
    assert abs(mean_n - paper_numbers["mean_n_shrink"]["value"]) < 0.25


def test_digits_at_large_stage_count(paper_numbers):
    """Abstract / Sec. 2.2: with Q <= 10 L^2, L = 10^4 stages keep at least 7 of 16 digits,
    and the extent 0.33 L^2 beta_RK2 over L evaluations is an acceleration above 6000."""
    g = paper_numbers["digits_kept_at_1e4_stages"]
    L = g["stages"]
    lost = math.log10(paper_numbers["q_practical_bound_factor"]["value"] * L * L)
    assert g["precision_digits"] - lost >= g["value"]
    c = frkc2_coeffs(400, 0.01)
    ratio = c.beta / (2.0 * 400 * 400)
    # explicit RK2 advances beta_RK2 = 2 per 2 evaluations; FRKC2 advances ratio*2L^2 per L
    accel = (ratio * 2 * L * L / L) / (2.0 / 2.0)
    assert accel > paper_numbers["acceleration_factor"]["value"]


def test_rejects_bad_arguments():
    for s in (0, 3, 516):
        with pytest.raises(ValueError):
            frkc2_coeffs(s)
    with pytest.raises(ValueError):
        frkc2_coeffs(8, 1.0)
