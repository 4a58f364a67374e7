"""The forward model as a differentiable torch operation.

``PtychoLoss.apply(obj, probe, positions, weights, I_meas, plan)`` returns the scalar
loss (float64). The forward runs the library's fused forward + adjoint once, so the
backward only scales the stored gradients by the incoming gradient. What is kept for
the backward is parameter-sized (object, probe, positions, weights), never
activation-sized: the per-position exit waves of a multislice model stay inside the
library's per-workgroup scratch (stored or recomputed, see ``Plan`` tune option
``recompute``), so memory is bounded by the number of workgroups, not by the number
of positions.
"""
from __future__ import annotations

from typing import Optional

import torch

from .ptyhip import Plan

_NAMES = ("obj", "probe", "pos", "weights")


class PtychoLoss(torch.autograd.Function):
    """Loss of Eq. (1) (or the Poisson loss) with gradients from the library adjoint.

    Gradients follow torch's convention for complex inputs (dL/dRe + i dL/dIm)."""

    @staticmethod
    def forward(ctx, obj, probe, positions, weights, I_meas, plan: Plan, plain: bool = False):
        needs = ctx.needs_input_grad
        grads = [n for n, f in zip(_NAMES, needs[:4]) if f]
        if weights is None and "weights" in grads:
            grads.remove("weights")
        args = (obj.detach(), probe.detach(), positions.detach(), I_meas.detach())
        w = None if weights is None else weights.detach()
        if not grads:
            loss = plan.forward(*args, weights=w)
            ctx.names = ()
            return loss.reshape(())
        out = plan.forward_adjoint(*args, weights=w, grads=grads, plain=plain)
        ctx.names = tuple(grads)
        ctx.save_for_backward(*[out["g_" + ("pos" if g == "pos" else g)] for g in grads])
        return out["loss"].reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        saved = dict(zip(ctx.names, ctx.saved_tensors))
        s = grad_out.to(torch.float32)
        res = []
        for n in _NAMES:
            g = saved.get(n)
            res.append(None if g is None else g * s)
        return (*res, None, None, None)


def ptycho_loss(obj, probe, positions, I_meas, plan: Plan, weights: Optional[torch.Tensor] = None,
                plain: bool = False):
    """Functional form of ``PtychoLoss``."""
    return PtychoLoss.apply(obj, probe, positions, weights, I_meas, plan, plain)
