"""CPU oracle for the FRKC2 superstep (O'Sullivan, arXiv:1702.03818).

TEST INFRASTRUCTURE. Only tests/, the smoke check and the benchmark's CPU
baseline import, call or link anything in this package. It is independent of
the GPU library: the two share no code, headers, tables or constants.

  coeffs.py  stepsizes (roots, damping, real extent, stage order), 50-digit mpmath + FP64
  stage.c    plain stage loops, adjoint and Gershgorin bound (gcc, FP64)
  stage.py   ctypes wrapper of stage.c (also the embedded first-order solution of Sec. 3)
  adaptive.py  error-controlled integration of Sec. 3: error norm, accept/reject,
             predictive controller, stage-count choice
  dense.py   dense matrix-polynomial brute force on tiny grids

Pins: every function is checked against closed forms, brute force or the
paper's printed numbers by the CPU tests, with one exception. The exact stage
permutation of greedy_order cannot be compared with the paper's own
coefficient table, which is not available: that permutation is "parity
unpinned"; its invariants (Q <= 10 L^2, mean n near 1.5) are pinned.
"""
from .coeffs import Coeffs, frkc2_coeffs, realised_q, stability_poly  # noqa: F401
from . import stage  # noqa: F401
