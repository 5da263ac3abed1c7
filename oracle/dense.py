"""Dense brute force on tiny grids: the superstep as a matrix polynomial.

TEST INFRASTRUCTURE (imported only by the tests).

For a linear operator f(w) = A w the superstep is exactly w^{n+1} = R(T A) w^n
with R(x) = prod_l (1 + a_l x) (Sec. 2, the stability polynomial determined by
w^{n+1} = R(TA) w^n). A is assembled here as an explicit matrix, face by face,
independently of the stencil loop in stage.c; since A is symmetric,
R(TA) = V diag(R(T lambda)) V^T with (lambda, V) from numpy.linalg.eigh, and
R(T lambda) is evaluated in 50-digit arithmetic so that no internal
amplification enters the brute-force result.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


def assemble(prob, D=None) -> np.ndarray:
    """Matrix of the linear operator (Laplace or variable coefficient) on prob's grid."""
    nx, ny, nz = (int(v) for v in prob.n)
    N = nx * ny * nz
    A = np.zeros((N, N))
    Dv = (D if D is not None else prob.D)
    Dv = None if Dv is None else np.asarray(Dv, dtype=np.float64).reshape(-1)
    inv_h2 = 1.0 / (prob.h * prob.h)
    dims = [nx, ny, nz][:prob.ndim]

    def flat(i):
        return i[0] + nx * (i[1] + ny * i[2])

    for p in range(N):
        i = [p % nx, (p // nx) % ny, p // (nx * ny)]
        for d in range(prob.ndim):
            for step in (-1, 1):
                j = list(i)
                j[d] += step
                ghost = False
                if j[d] < 0 or j[d] >= dims[d]:
                    if prob.bc == 1:
                        ghost = True
                    else:
                        j[d] %= dims[d]
                if prob.op == 0:
                    Df = prob.d_const
                else:
                    Df = Dv[p] if ghost else 0.5 * (Dv[p] + Dv[flat(j)])
                A[p, p] -= Df * inv_h2
                if not ghost:
                    A[p, flat(j)] += Df * inv_h2
    return A


def R_hp(a: np.ndarray, x: float) -> float:
    """R(x) for real x, in 50-digit arithmetic from the FP64 stepsizes."""
    with mp.workdps(50):
        r = mp.mpc(1)
        xm = mp.mpf(float(x))
        for al in a:
            r *= 1 + mp.mpc(float(al.real), float(al.imag)) * xm
        return float(mp.re(r))


def R_hp_complex(a: np.ndarray, z: complex) -> complex:
    """R(z) for complex z, in 50-digit arithmetic from the FP64 stepsizes."""
    with mp.workdps(50):
        r = mp.mpc(1)
        zm = mp.mpc(float(z.real), float(z.imag))
        for al in a:
            r *= 1 + mp.mpc(float(al.real), float(al.imag)) * zm
        return complex(r)


def superstep(prob, w, a: np.ndarray, T: float, D=None) -> np.ndarray:
    """R(T A) w via the eigendecomposition of the assembled symmetric A."""
    A = assemble(prob, D)
    lam, V = np.linalg.eigh(A)
    r = np.array([R_hp(a, T * l) for l in lam])
    return V @ (r * (V.T @ np.asarray(w, dtype=np.float64).reshape(-1)))
