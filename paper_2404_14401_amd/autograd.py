"""torch.autograd.Function over the GPU adjoint: gradients of the final-state
infidelity (or energy) of a batch of condensates with respect to their lattice-depth
controls.

Forward runs the real-time split step on every member with the given knot values and
returns the per-member losses; when the knots need a gradient the same call also runs
the discrete adjoint's reverse sweep (reusing the forward's final state), whose result
backward returns.  A loss-only evaluation (no_grad, or knots without requires_grad)
runs the forward sweep alone."""
from __future__ import annotations

import numpy as np
import torch

from . import gpe


class GPEControl(torch.autograd.Function):
    """loss = GPEControl.apply(knots, batch, psi0s, targets, nsteps, t0, mode, control, loss)

    knots: float64 tensor (n, M) of lattice depth values (host or device) for the x
    lattice (control "x") or the pump, y lattice (control "pump");
    psi0s, targets: lists of n complex64 CUDA tensors (ny, nx) (targets None for the
    energy loss)."""

    @staticmethod
    def forward(ctx, knots, batch, psi0s, targets, nsteps, t0=0.0, mode="auto", control="x", loss="fidelity"):
        k = knots.detach().to("cpu", torch.float64).numpy()
        want = bool(ctx.needs_input_grad[0])
        loss, grad, info = gpe.adjoint(batch, psi0s, targets, nsteps, k, t0=t0, mode=mode, control=control,
                                       loss=loss, want_grad=want)
        if want:
            ctx.save_for_backward(torch.from_numpy(grad).to(knots.device))
        ctx.info = info
        return torch.from_numpy(loss).to(knots.device)

    @staticmethod
    def backward(ctx, gloss):
        (grad,) = ctx.saved_tensors
        return gloss[:, None].to(grad.dtype) * grad, None, None, None, None, None, None, None, None


def control_loss(knots, batch, psi0s, targets, nsteps, t0=0.0, mode="auto", control="x", loss="fidelity"):
    return GPEControl.apply(knots, batch, psi0s, targets, nsteps, t0, mode, control, loss)


__all__ = ["GPEControl", "control_loss", "np"]
