"""torch.autograd.Function over the FRKC2 superstep and its adjoint.

superstep_fn(u0, logD, grid, T, s, nsteps) advances u0 by nsteps supersteps
of the variable-coefficient diffusion u_t = div(D grad u), D = exp(logD), on
the GPU and returns w(nsteps T). Its backward returns dJ/du0 and dJ/dlogD.

Two ways to keep what the backward needs, with the same bits:

* stage store (store_stages=True): the forward runs frkc2_step_store, which
  keeps each superstep's s complex stage states (16 s bytes per point and
  superstep), and the backward runs frkc2_step_adjoint_stored on them, the
  transposed stages in reverse order (lam <- lam + conj(tau_l) A lam),
  accumulating D * dJ/dD;
* checkpoints (store_stages=False): the forward keeps one real state per
  superstep (8 bytes per point) and the backward's frkc2_step_adjoint
  recomputes each superstep's stages from it before the reverse stages.

store_stages=None takes the store when all of it fits in a quarter of the
device memory free at the forward's start. The derivative arithmetic is all in
the library's kernels; this module only orders the calls and owns the buffers.
"""
from __future__ import annotations

import torch

from . import frkc2 as F

STORE_FRACTION = 0.25   # share of the free device memory the automatic stage store may take


def _want_store(grid, s, nsteps, device):
    per = F.frkc2_workspace_bytes(grid, s, F.WS_STAGES)
    free, _ = torch.cuda.mem_get_info(device)
    return per > 0 and nsteps * per <= STORE_FRACTION * free


class FRKC2Superstep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, logD, grid, T, s, nsteps, nu, store_stages):
        if u0.dtype != torch.float64 or logD.dtype != torch.float64:
            raise TypeError("superstep_fn works in float64")
        D = torch.exp(logD.detach()).contiguous()
        w = u0.detach().contiguous().clone()
        nsteps, s = int(nsteps), int(s)
        store = _want_store(grid, s, nsteps, w.device) if store_stages is None else bool(store_stages)
        saved = []
        for _ in range(nsteps):
            if store:
                st = F.stage_store(grid, s, device=w.device)
                F.frkc2_step_store(grid, w, D, float(T), s, st, nu=float(nu))
                saved.append(st)
            else:
                saved.append(w.clone())
                F.frkc2_step(grid, w, D, T=float(T), s=s, nu=float(nu), nsteps=1)
        ctx.grid, ctx.T, ctx.s, ctx.nu, ctx.store = grid, float(T), s, float(nu), store
        ctx.save_for_backward(D, *saved)
        return w

    @staticmethod
    def backward(ctx, grad_w):
        D, *saved = ctx.saved_tensors
        lam = grad_w.detach().contiguous().clone()
        lam_n = torch.empty_like(lam)
        g_logD = torch.zeros_like(D)
        for item in reversed(saved):
            if ctx.store:
                F.frkc2_step_adjoint_stored(ctx.grid, item, D, ctx.T, ctx.s, lam, lam_n, g_logD,
                                            nu=ctx.nu)
            else:
                F.frkc2_step_adjoint(ctx.grid, item, D, ctx.T, ctx.s, lam, lam_n, g_logD, nu=ctx.nu)
            lam, lam_n = lam_n, lam
        return lam, g_logD, None, None, None, None, None, None


def superstep_fn(u0, logD, grid, T, s, nsteps=1, nu=0.01, store_stages=None):
    """w after nsteps FRKC2 supersteps of length T with s stages (differentiable in u0, logD).
    store_stages: True keeps every stage state for the backward, False keeps one checkpoint
    per superstep and recomputes, None chooses by free device memory."""
    return FRKC2Superstep.apply(u0, logD, grid, T, s, nsteps, nu, store_stages)
