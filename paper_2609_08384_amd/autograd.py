"""torch.autograd.Function around the engine's hand-written adjoint.

ssfm(fields, params, nsteps, dk=None, checkpoint_every=20) propagates the
complex64 CUDA fields nsteps z-steps from z = 0 with the HIP engine and
returns the output fields; backpropagating through them runs the engine's
reverse sweep (brahms_adjoint_backward), giving gradients with respect to the
input fields and, when `dk` is a float64 tensor, the per-step phase-mismatch
profile.  Complex gradients follow PyTorch's convention dJ/dRe + i dJ/dIm.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import brahms


class _SSFM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, nsteps, every, pass_order, dk, *fields):
        nt, ny, nx = fields[0].shape
        p = brahms.Params(dz=params.dz, fields=params.fields, dk_const=params.dk_const,
                          dk=None if dk is None else [float(v) for v in dk.detach().cpu()],
                          dx=params.dx, dy=params.dy, dt=params.dt)
        work = [f.detach().to(torch.complex64).contiguous().clone() for f in fields]
        plan = brahms.Plan(nx, ny, nt, len(fields), p)
        if pass_order is not None:
            plan.set_schedule(pass_order)
        plan.bind(work)
        plan.adjoint_forward(nsteps, every)
        ctx.plan = plan
        ctx.dk_meta = None if dk is None else (dk.dtype, dk.device)
        return tuple(work)

    @staticmethod
    def backward(ctx, *grad_out):
        plan = ctx.plan
        grads = []
        for g, f in zip(grad_out, plan.fields):
            if g is None:
                grads.append(torch.zeros_like(f))
            else:
                grads.append(g.detach().to(torch.complex64).contiguous().clone())
        gdk = plan.adjoint_backward(grads)
        ctx.plan = None
        dk_grad = None
        if ctx.dk_meta is not None:
            dk_grad = torch.as_tensor(gdk, dtype=ctx.dk_meta[0], device=ctx.dk_meta[1])
        return (None, None, None, None, dk_grad, *grads)


def ssfm(fields: Sequence[torch.Tensor], params: brahms.Params, nsteps: int,
         dk: Optional[torch.Tensor] = None, checkpoint_every: int = 20,
         pass_order: Optional[int] = None):
    """Differentiable propagation from z = 0 (see the module doc)."""
    return _SSFM.apply(params, int(nsteps), int(checkpoint_every), pass_order, dk, *fields)
