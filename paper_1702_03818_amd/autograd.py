"""torch.autograd.Function over the FRKC2 superstep and its adjoint.

superstep_fn(u0, logD, grid, T, s, nsteps) advances u0 by nsteps supersteps
of the variable-coefficient diffusion u_t = div(D grad u), D = exp(logD), on
the GPU and returns w(nsteps T). Its backward returns dJ/du0 and dJ/dlogD.

Forward keeps one checkpoint per superstep (the real state w_n, 8 bytes per
point). Backward walks the supersteps in reverse; for each it calls
frkc2_step_adjoint, which recomputes the superstep's s complex stages from
w_n into its workspace and runs the transposed stages in reverse order
(lam <- lam + conj(tau_l) A lam), accumulating D * dJ/dD. The derivative
arithmetic is all in the library's kernels; this module only orders the
calls and owns the checkpoints.
"""
from __future__ import annotations

import torch

from . import frkc2 as F


class FRKC2Superstep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, logD, grid, T, s, nsteps, nu):
        if u0.dtype != torch.float64 or logD.dtype != torch.float64:
            raise TypeError("superstep_fn works in float64")
        D = torch.exp(logD.detach()).contiguous()
        w = u0.detach().contiguous().clone()
        ckpts = []
        for _ in range(int(nsteps)):
            ckpts.append(w.clone())
            F.frkc2_step(grid, w, D, T=float(T), s=int(s), nu=float(nu), nsteps=1)
        ctx.grid, ctx.T, ctx.s, ctx.nu = grid, float(T), int(s), float(nu)
        ctx.save_for_backward(D, *ckpts)
        return w

    @staticmethod
    def backward(ctx, grad_w):
        D, *ckpts = ctx.saved_tensors
        lam = grad_w.detach().contiguous().clone()
        lam_n = torch.empty_like(lam)
        g_logD = torch.zeros_like(D)
        for w_n in reversed(ckpts):
            F.frkc2_step_adjoint(ctx.grid, w_n, D, ctx.T, ctx.s, lam, lam_n, g_logD, nu=ctx.nu)
            lam, lam_n = lam_n, lam
        return lam, g_logD, None, None, None, None, None


def superstep_fn(u0, logD, grid, T, s, nsteps=1, nu=0.01):
    """w after nsteps FRKC2 supersteps of length T with s stages (differentiable in u0, logD)."""
    return FRKC2Superstep.apply(u0, logD, grid, T, s, nsteps, nu)
