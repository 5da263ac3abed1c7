"""FRKC2 superstep on AMD MI355X (gfx950): HIP kernels behind a C ABI.

O'Sullivan, "Factorized Runge-Kutta-Chebyshev Methods", arXiv:1702.03818.
The library (libfrkc2.so, built in-tree by paper_1702_03818_amd.build) holds
the stepsize generator and the GPU kernels; this package is its binding:

  frkc2        ctypes binding with the C names (frkc2_coeffs, frkc2_step, ...)
  autograd     torch.autograd.Function over frkc2_step / frkc2_step_adjoint
  workloads    seeded synthetic inputs (no method arithmetic)
  build        compiles the library for gfx950
"""
from . import frkc2  # noqa: F401  (loads the shared library lazily, on first call)
from .frkc2 import (frkc2_coeffs, frkc2_step, frkc2_step_adjoint, frkc2_step_batched,  # noqa: F401
                    frkc2_rho_bound, frkc2_reduce, frkc2_workspace_bytes)
