"""Seeded synthetic inputs for the FRKC2 superstep.

This module only draws inputs: grids, diffusivity fields, initial states and
targets. It holds none of the method's arithmetic (no stepsizes, no stencil,
no stage loop), so the GPU library and the CPU oracle can both be fed from it
without sharing any computation.

Arrays are float64, C-ordered with shape (nz, ny, nx) (x fastest in memory),
which is the flat layout index = x + nx*(y + ny*z) the library expects.

Workloads (seeded numpy PCG64; the recipe is stated next to each generator):
  heat1d        1D u_t = u_xx, periodic, N = 1024, sum of 8 sine modes
  diffusion3d   3D u_t = div(D grad u), 256^3, Dirichlet zero, lognormal D
  porous2d      2D u_t = div(u^2 grad u), 4096^2, periodic
  batched       512 independent 2D/3D variable-D problems of uneven size and s
  adjoint3d     3D variable-D problem, 128^3, with a seeded target field
  brusselator   2D two-species Brusselator, 200^2, periodic (the paper's default user
                problem, Sec. 3.1; its initial data are fixed, no random draw)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BC_PERIODIC = 0
BC_DIRICHLET0 = 1
OP_LAPLACE = 0
OP_VARCOEF = 1
OP_POROUS2 = 2
OP_BRUSS2 = 3
OP_ADVDIFF = 4


@dataclass
class Problem:
    ndim: int
    n: tuple            # (nx, ny, nz) with unused dimensions 1
    h: float            # grid spacing, equal in every dimension
    bc: int
    op: int
    d_const: float = 1.0
    D: np.ndarray | None = None     # cell diffusivity (op = OP_VARCOEF)
    w0: np.ndarray | None = None    # initial state
    meta: dict = field(default_factory=dict)
    vel: tuple = (0.0, 0.0, 0.0)    # advection velocity per dimension (op = OP_ADVDIFF)

    @property
    def nfield(self) -> int:
        """Values per grid point (the Brusselator stores v, then w)."""
        return 2 if self.op == OP_BRUSS2 else 1

    @property
    def shape(self):
        nx, ny, nz = self.n
        s = {1: (nx,), 2: (ny, nx), 3: (nz, ny, nx)}[self.ndim]
        return (2,) + s if self.nfield == 2 else s

    @property
    def npoints(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def nstate(self) -> int:
        return self.nfield * self.npoints


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _nodes(n: int, bc: int) -> tuple[np.ndarray, float]:
    """Node coordinates on [0, 1]: periodic x_i = i/n; Dirichlet x_i = (i+1)/(n+1)."""
    if bc == BC_PERIODIC:
        h = 1.0 / n
        return np.arange(n) * h, h
    h = 1.0 / (n + 1)
    return (np.arange(n) + 1) * h, h


def smooth_field(shape, sigma_cells: float, rng) -> np.ndarray:
    """White N(0,1) noise smoothed by a periodic Gaussian of sigma_cells, re-standardised."""
    g = rng.standard_normal(shape)
    G = np.fft.rfftn(g)
    k2 = np.zeros(G.shape)
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = np.fft.rfftfreq(n)
        else:
            k = np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[ax] = len(k)
        k2 = k2 + (k.reshape(sh) * 2 * np.pi) ** 2
    G *= np.exp(-0.5 * sigma_cells ** 2 * k2)
    out = np.fft.irfftn(G, s=shape, axes=tuple(range(len(shape))))
    out -= out.mean()
    sd = out.std()
    return out / sd if sd > 0 else out


def lognormal_D(shape, sigma_cells: float, rng) -> np.ndarray:
    """D = exp(g), g a standardised smooth field, so log D ~ N(0, 1) pointwise."""
    return np.ascontiguousarray(np.exp(smooth_field(shape, sigma_cells, rng)))


def blobs(shape, coords, count: int, rng, radii=(0.03, 0.08), amps=(0.5, 1.5),
          centres=(0.2, 0.8)) -> np.ndarray:
    """Sum of `count` isotropic Gaussian blobs, centres U[centres]^d, radii and amplitudes uniform.

    coords lists the node coordinates per array axis (same order as shape).
    """
    out = np.zeros(shape)
    d = len(shape)
    for _ in range(count):
        c = rng.uniform(centres[0], centres[1], size=d)
        r = rng.uniform(radii[0], radii[1])
        a = rng.uniform(amps[0], amps[1])
        term = np.array(a)
        for ax in range(d):
            g1 = np.exp(-0.5 * ((coords[ax] - c[ax]) / r) ** 2)
            sh = [1] * d
            sh[ax] = shape[ax]
            term = term * g1.reshape(sh)
        out += term
    return out


def heat1d(seed: int = 1, N: int = 1024) -> Problem:
    """1D heat u_t = u_xx on [0, 1) periodic, h = 1/N, u0 = sum_{k=1..8} A_k sin(2 pi k x), A_k ~ N(0, 1)."""
    rng = _rng(seed)
    A = rng.standard_normal(8)
    x, h = _nodes(N, BC_PERIODIC)
    u0 = np.zeros(N)
    for k in range(1, 9):
        u0 += A[k - 1] * np.sin(2 * np.pi * k * x)
    return Problem(1, (N, 1, 1), h, BC_PERIODIC, OP_LAPLACE, 1.0, None, u0,
                   meta={"amplitudes": A, "modes": np.arange(1, 9)})


def diffusion3d(seed: int = 2, n: int = 256, nblobs: int = 16, sigma_cells: float = 4.0,
                n_xyz=None) -> Problem:
    """3D u_t = div(D grad u), n^3 interior nodes, Dirichlet zero, h = 1/(n+1).

    D = exp(g), g white noise smoothed with a Gaussian of sigma_cells cells and
    re-standardised (lognormal, sigma 1). u0 = nblobs Gaussian blobs with
    centres U[0.2, 0.8]^3, radii U[0.03, 0.08], amplitudes U[0.5, 1.5].
    n_xyz overrides the cube with an (nx, ny, nz) box (parity cases).
    """
    rng = _rng(seed)
    nx, ny, nz = n_xyz if n_xyz is not None else (n, n, n)
    shape = (nz, ny, nx)
    D = lognormal_D(shape, sigma_cells, rng)
    xs, h = _nodes(nx, BC_DIRICHLET0)
    ys, _ = _nodes(ny, BC_DIRICHLET0)
    zs, _ = _nodes(nz, BC_DIRICHLET0)
    if not (nx == ny == nz):
        h = 1.0 / (max(nx, ny, nz) + 1)
        xs, ys, zs = (np.arange(nx) + 1) * h, (np.arange(ny) + 1) * h, (np.arange(nz) + 1) * h
    u0 = blobs(shape, (zs, ys, xs), nblobs, rng)
    return Problem(3, (nx, ny, nz), h, BC_DIRICHLET0, OP_VARCOEF, 1.0, D, u0)


def porous2d(seed: int = 3, n: int = 4096, sigma_cells: float = 64.0) -> Problem:
    """2D u_t = div(u^2 grad u), n^2 periodic, h = 1/n, u0 = 1 + 0.5 g / max|g| in [0.5, 1.5]."""
    rng = _rng(seed)
    g = smooth_field((n, n), sigma_cells, rng)
    u0 = 1.0 + 0.5 * g / np.abs(g).max()
    return Problem(2, (n, n, 1), 1.0 / n, BC_PERIODIC, OP_POROUS2, 1.0, None,
                   np.ascontiguousarray(u0))


def _batch_draw(rng, side2d, side3d, m_range):
    """Dimension, side and M of one batched problem: the first draws of its generator."""
    dim = 2 if rng.random() < 0.5 else 3
    lo, hi = side2d if dim == 2 else side3d
    side = int(rng.integers(lo, hi + 1))
    M = int(rng.integers(m_range[0], m_range[1] + 1))
    return dim, side, M


def batched_shapes(seed: int = 4, count: int = 512, side2d=(32, 512), side3d=(32, 128),
                   m_range=(4, 100)) -> list[tuple[Problem, int]]:
    """The problems of batched() without their fields (D and u0 left None): the grids and
    stage counts only, for host-side checks that need no data."""
    out = []
    for child in np.random.SeedSequence(seed).spawn(count):
        rng = np.random.Generator(np.random.PCG64(child))
        dim, side, M = _batch_draw(rng, side2d, side3d, m_range)
        _, h = _nodes(side, BC_DIRICHLET0)
        n = (side, side, side) if dim == 3 else (side, side, 1)
        out.append((Problem(dim, n, h, BC_DIRICHLET0, OP_VARCOEF, 1.0, None, None), 2 * M))
    return out


def batched(seed: int = 4, count: int = 512, side2d=(32, 512), side3d=(32, 128),
            m_range=(4, 100)) -> list[tuple[Problem, int]]:
    """`count` independent Dirichlet variable-D problems and their stage counts.

    Per problem (child seeds from SeedSequence(seed).spawn): dimension 2 or 3
    with probability 1/2; side uniform on side2d (2D) or side3d (3D) inclusive;
    s = 2M with M uniform on m_range inclusive; D lognormal as in diffusion3d
    with sigma = max(2, side/32) cells; u0 = 4 Gaussian blobs.
    """
    out = []
    for child in np.random.SeedSequence(seed).spawn(count):
        rng = np.random.Generator(np.random.PCG64(child))
        dim, side, M = _batch_draw(rng, side2d, side3d, m_range)
        shape = (side,) * dim
        D = lognormal_D(shape, max(2.0, side / 32.0), rng)
        xs, h = _nodes(side, BC_DIRICHLET0)
        u0 = blobs(shape, (xs,) * dim, 4, rng)
        n = (side, side, side) if dim == 3 else (side, side, 1)
        out.append((Problem(dim, n, h, BC_DIRICHLET0, OP_VARCOEF, 1.0, D, u0), 2 * M))
    return out


def adjoint3d(seed: int = 5, n: int = 128, nblobs: int = 8) -> tuple[Problem, np.ndarray]:
    """diffusion3d-style problem (n^3, Dirichlet, lognormal D, 8 blobs) plus an independent blob target."""
    rng = _rng(seed)
    shape = (n, n, n)
    D = lognormal_D(shape, 4.0, rng)
    xs, h = _nodes(n, BC_DIRICHLET0)
    u0 = blobs(shape, (xs, xs, xs), nblobs, rng)
    target = blobs(shape, (xs, xs, xs), nblobs, rng)
    return Problem(3, (n, n, n), h, BC_DIRICHLET0, OP_VARCOEF, 1.0, D, u0), target


def random_state(shape, seed: int, smooth: float | None = None) -> np.ndarray:
    """A seeded test field: white N(0,1) or, with smooth, a standardised smooth field."""
    rng = _rng(seed)
    if smooth is None:
        return rng.standard_normal(shape)
    return smooth_field(shape, smooth, rng)


def brusselator(n: int = 200, d: float = 0.02) -> Problem:
    """Sec. 3.1's two-species Brusselator on the periodic unit square, n x n cells at
    x_i = i/n: v0 = 1 + sin(2 pi x), w0 = 3 + cos(2 pi y); diffusion d = 0.02 (spectral
    radius about 8 d n^2 = 6400 at n = 200). State: v then w, each (n, n) with x fastest."""
    x = np.arange(n) / n
    X = x[None, :]
    Y = x[:, None]
    v0 = np.broadcast_to(1.0 + np.sin(2 * np.pi * X), (n, n))
    w0 = np.broadcast_to(3.0 + np.cos(2 * np.pi * Y), (n, n))
    p = Problem(2, (n, n, 1), 1.0 / n, BC_PERIODIC, OP_BRUSS2, d)
    p.w0 = np.ascontiguousarray(np.stack([v0, w0]))
    p.meta = {"A": 1.0, "B": 3.0}
    return p
