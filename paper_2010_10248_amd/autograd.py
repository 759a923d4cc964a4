"""torch.autograd wrappers of the library's linear modelling map and misfit
gradient (argument marshalling only: every step runs in the HIP library).

* ``modelling(q, prop)``: traces d = F q of the wavelets q [nt][nsrc] for a
  fixed model; backward applies the exact adjoint F^T (tb_adjoint).
* ``misfit(m, shot, d_obs)``: J(m) = 1/2 sum |P_r u^k - d_obs^k|^2 for the
  squared slowness m [nx][ny][nz]; backward returns dJ/dm from the
  checkpointed adjoint gradient (tb_gradient), computed together with J.
"""
from __future__ import annotations

import numpy as np
import torch

from . import tb


class _Modelling(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, prop, sched):
        ctx.prop, ctx.sched = prop, sched
        ws = prop.workspace(sched, tb.OP_FORWARD)
        d = torch.empty((prop.shot.nt, prop.nrec), dtype=torch.float32, device=q.device)
        # The wavelets are baked into the sparse handle by the inspector, so a
        # new q needs a new inspection of the same coordinates.
        sp = tb.inspect_sparse(prop.model, prop.shot.src_xyz, q.detach().double().cpu().numpy(),
                               prop.shot.rec_xyz)
        try:
            tb.forward(prop.model, sp, sched, ws, d)
            torch.cuda.current_stream().synchronize()
        finally:
            tb.destroy_sparse(sp)
        return d

    @staticmethod
    def backward(ctx, gd):
        return ctx.prop.adjoint(gd.float().contiguous(), ctx.sched), None, None


def modelling(q: torch.Tensor, prop: "tb.Acoustic", sched=None) -> torch.Tensor:
    return _Modelling.apply(q, prop, sched)


class _Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, shot, d_obs, sched, checkpoint_every, damp_vmax):
        prop = tb.Acoustic(shot, slowness2=m.detach(), device=m.device, damp_vmax=damp_vmax)
        try:
            J, g = prop.gradient(d_obs.float().contiguous(), sched, checkpoint_every)
        finally:
            prop.close()
        ctx.save_for_backward(g)
        return torch.tensor(J, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        return (gJ.to(g.dtype) * g), None, None, None, None, None


def misfit(m: torch.Tensor, shot, d_obs: torch.Tensor, sched=None, checkpoint_every: int = 0,
           damp_vmax: float = 0.0) -> torch.Tensor:
    """J(m) as a float64 scalar tensor. The library takes m itself (c = dt^2/m
    in FP64, rounded once). The damping profile is held fixed, as the
    gradient assumes: its velocity is damp_vmax, or when that is 0 the
    largest vp of the shot's own model (not of m)."""
    if not damp_vmax > 0.0:
        damp_vmax = float(np.max(shot.vp))
    return _Misfit.apply(m, shot, d_obs, sched, checkpoint_every, damp_vmax)
