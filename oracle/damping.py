"""Oracle for the damping a problem with a small hyperbolic part needs (Sec. 2.1, "Damping").

TEST INFRASTRUCTURE. Only the tests may import this module.

Sec. 2.1 says two things about damping: it scales the marginally stable maxima of |R| on the
real axis down by about (1 - nu0) while the real extent shrinks by about (1 - nu), and it makes
the scheme usable on problems whose spectrum leaves the real axis a little (advection-diffusion
with Peclet numbers up to about 10, where the paper observes a 25 % loss of extent). The paper
does not say how much damping a given problem needs, nor what its Peclet number is measured
on.

Reading used here. The operator is the library's advection-diffusion operator: constant
diffusivity d and velocity v, central differences written face by face, the face toward -x_k
with coefficient d + v_k h/2 and the face toward +x_k with d - v_k h/2. On a periodic grid of
n_k cells per axis its eigenvectors are the Fourier modes, with eigenvalues

    lambda(theta) = sum_k [ (d + v_k h/2)(e^{-i theta_k} - 1) + (d - v_k h/2)(e^{i theta_k} - 1) ] / h^2,
    theta_k = 2 pi j_k / n_k,

so a superstep of length T is stable when |R(T lambda)| <= 1 for every mode. The library runs
at T = betabar(nu) / rho, rho the Gershgorin bound (|sum_f c_f| + sum_f |c_f|) / h^2; the
damping the problem needs is the smallest nu of a grid (0, 0.01, 0.02, ...) for which every
mode passes at that T. The Peclet number is v L / d with L = n h the period.
"""
from __future__ import annotations

import numpy as np

from .coeffs import frkc2_coeffs


def face_coeffs(h: float, d: float, vel) -> list:
    """(c_minus, c_plus) per axis: the coefficients of the faces toward -x_k and +x_k."""
    return [(d + 0.5 * h * v, d - 0.5 * h * v) for v in vel]


def symbols(n, h: float, d: float, vel) -> np.ndarray:
    """Eigenvalues of the periodic operator, one per Fourier mode (all prod(n) of them)."""
    lam = np.zeros(1, dtype=complex)
    for nk, (cm, cp) in zip(n, face_coeffs(h, d, vel)):
        th = 2.0 * np.pi * np.arange(nk) / nk
        lk = (cm * (np.exp(-1j * th) - 1.0) + cp * (np.exp(1j * th) - 1.0)) / (h * h)
        lam = (lam[:, None] + lk[None, :]).reshape(-1)
    return lam


def gershgorin(h: float, d: float, vel) -> float:
    """rho = (|sum of face coefficients| + sum of their moduli) / h^2."""
    cs = [c for pair in face_coeffs(h, d, vel) for c in pair]
    return (abs(sum(cs)) + sum(abs(c) for c in cs)) / (h * h)


def log_amplification(a: np.ndarray, z: np.ndarray) -> np.ndarray:
    """log |R(z)| = sum_l log |1 + a_l z| for each z."""
    out = np.zeros(z.shape)
    for al in a:
        out += np.log(np.abs(1.0 + al * z))
    return out


def min_damping(n, h: float, d: float, vel, s: int, nu_max: float = 0.6, step: float = 0.01,
                tol: float = 1e-12):
    """Smallest nu = step * j <= nu_max with max |R(T lambda)| <= 1 + tol over every mode at
    T = betabar(nu) / rho. Returns a dict with nu, the real extents beta(nu) and beta(0), the
    length T and the largest log |R| over the modes, or None if no nu of the grid passes."""
    lam = symbols(n, h, d, vel)
    rho = gershgorin(h, d, vel)
    beta0 = frkc2_coeffs(s, 0.0).beta
    for j in range(int(round(nu_max / step)) + 1):
        nu = round(j * step, 10)
        c = frkc2_coeffs(s, nu)
        T = c.beta_bar / rho
        worst = float(log_amplification(c.a, T * lam).max())
        if worst <= np.log1p(tol):
            return {"nu": nu, "beta": c.beta, "beta0": beta0, "T": T, "log_amp": worst,
                    "coeffs": c}
    return None
