"""torch.autograd wrapper: forward modelling whose backward is the adjoint reverse pass.

Forward = smi_forward with boundary saving (Sec. 4.2): the bands and the final wavefield are
kept in the call's workspace instead of the wavefield history.  Backward = smi_adjoint_
reconstruct with the incoming gradient dL/d(dcal) as adjoint source (eq. 8): the source field
is rebuilt backwards from the bands while the adjoint field is propagated, and the result is
dL/dVp with the density held fixed (eq. 7 with kappa = rho Vp^2) and, when the density requires
a gradient, dL/drho with Vp held fixed (the parametrisation family 1 of Sec. 2.2).  For L = 1/2 dt sum (dcal -
dobs)^2 this is exactly the FWI gradient of eq. (6).
"""
from __future__ import annotations

import torch

from . import binding as B


class SmiForward(torch.autograd.Function):
    """dcal = F(vp, rho); vjp(g) = (dL/dVp at fixed rho, dL/drho at fixed Vp) from one reverse
    pass (the density gradient only when rho requires grad; stf is not differentiated)."""

    @staticmethod
    def forward(ctx, vp, rho, stf, grid, acq, smi_ctx, stream):
        dcal, _, state = smi_ctx.forward(grid, acq, vp.detach().contiguous(), rho.contiguous(),
                                         stf.contiguous(), save=True, stream=stream)
        ctx.state = state
        ctx.smi = smi_ctx
        ctx.stream = stream
        ctx.shape = vp.shape
        return dcal

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_dcal):
        state = ctx.state
        if state is None or state.consumed:
            raise RuntimeError("the saved forward pass was already consumed by a backward pass")
        want_rho = ctx.needs_input_grad[1]
        fam = ctx.smi.option(B.OPT_FAMILY, 1)
        if fam != 1:
            ctx.smi.set_option(B.OPT_FAMILY, 1)         # the inputs are (Vp, rho)
        try:
            out = ctx.smi.adjoint_reconstruct(state, grad_dcal.contiguous(), grad=True,
                                              grad_rho=want_rho, image=False, illum=False,
                                              stream=ctx.stream)
        finally:
            if fam != 1:
                ctx.smi.set_option(B.OPT_FAMILY, fam)
        ctx.state = None
        g_rho = out["grad_rho"].view(ctx.shape) if want_rho else None
        return out["grad"].view(ctx.shape), g_rho, None, None, None, None, None


def forward_modelling(vp, rho, stf, grid, acq, smi_ctx=None, stream=None):
    """Seismograms (flat, shot s at nt*rec_off[s], layout [nt][nrec_s]) with autograd support
    for vp.  The model speed range is taken from grid.vpmin / grid.vpmax when set."""
    smi_ctx = smi_ctx or B.context(vp.device.index or 0)
    return SmiForward.apply(vp, rho, stf, grid, acq, smi_ctx, stream)


def l2_misfit(dcal, dobs, dt: float):
    """eq. (6) with the rectangle rule: J = 1/2 dt sum (dcal - dobs)^2 (float64 sum)."""
    r = (dcal - dobs).double()
    return 0.5 * dt * torch.sum(r * r)
