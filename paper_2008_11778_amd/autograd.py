"""torch.autograd.Function around the forward map f(m) = R F(m).

forward() runs the HIP forward pass keeping wavefield checkpoints (every
``ckpt_every`` steps of the Context); backward() maps the incoming data-space
gradient through the exact discrete adjoint (recompute each segment from its
checkpoint, adjoint steps with zero-lag imaging, fold), so a long record's
memory is O(nt/k + k) wavefields and no second full forward is run.

If another forward run has used the same Context in between (the kept
checkpoints belong to a different model), backward() first re-runs the
forward for the saved model, so the result is always J'(m)^T grad_d.
"""
from __future__ import annotations

import torch

from ._lib import Context


class SeismicForward(torch.autograd.Function):
    @staticmethod
    def forward(fctx, m: torch.Tensor, context: Context):
        m_c = m.detach().contiguous()
        d = context.forward_model(m_c, keep_ckpt=True)
        fctx.context = context
        fctx.gen = context.generation
        fctx.save_for_backward(m_c)
        return d

    @staticmethod
    def backward(fctx, grad_d: torch.Tensor):
        (m_c,) = fctx.saved_tensors
        context = fctx.context
        if context.generation != fctx.gen:
            context.forward_model(m_c, keep_ckpt=True)
            fctx.gen = context.generation
        grad_m = context.adjoint_from_residual(grad_d.detach().contiguous())
        return grad_m, None


def seismic_forward(m: torch.Tensor, context: Context) -> torch.Tensor:
    """Differentiable f(m): [S][nt][R] seismograms from the model m [nz][nx]."""
    return SeismicForward.apply(m, context)


class Misfit(torch.autograd.Function):
    """J = 1/2 ||d - d_obs||^2 (eq. FWI) through the library's residual
    kernel (r = d - d_obs in FP32, J in FP64 in a fixed order, the same
    arithmetic as the C-ABI problem); the gradient with respect to d is r,
    scaled by the incoming gradient of J."""

    @staticmethod
    def forward(fctx, d: torch.Tensor, d_obs: torch.Tensor, context: Context):
        r, J = context.residual_misfit(d.detach().contiguous(), d_obs.contiguous())
        fctx.save_for_backward(r)
        return J.view(())

    @staticmethod
    def backward(fctx, grad_J: torch.Tensor):
        from ._lib import scale
        (r,) = fctx.saved_tensors
        return scale(float(grad_J.item()), r), None, None


def misfit(d: torch.Tensor, d_obs: torch.Tensor, context: Context) -> torch.Tensor:
    """Differentiable J(d) = 1/2 ||d - d_obs||^2 as a device FP64 scalar."""
    return Misfit.apply(d, d_obs, context)
