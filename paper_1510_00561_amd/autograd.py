"""Differentiable contourlet transform: torch.autograd wrappers over libct.

Gradients run on the device through the hand-written transposes of the C
ABI. The CT frame is not tight, so the transpose of the inverse is not the
forward transform:
  CTForward  y = F x   backward: gx = F^T gy   (ct_forward_adjoint)
  CTInverse  x = S c   backward: gc = S^T gx   (ct_inverse_adjoint)
  STQuant    c~ = dequantise(quantise(c))  backward: identity (straight through)

With these, encoder-side rate-distortion optimisation of the coefficients
runs on the GPU, e.g. minimising ||S Q(c) - x||^2 + lambda ||c||_1 over c.
"""
import torch

from . import ct as _ct


class CTForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.forward(x.contiguous())

    @staticmethod
    def backward(ctx, gy):
        return ctx.plan.forward_adjoint(gy.contiguous()), None


class CTInverse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, plan):
        ctx.plan = plan
        return plan.inverse(c.contiguous())

    @staticmethod
    def backward(ctx, gx):
        return ctx.plan.inverse_adjoint(gx.contiguous()), None


class STQuant(torch.autograd.Function):
    """Quantise and dequantise (the codec round trip); identity gradient."""

    @staticmethod
    def forward(ctx, c, steps, plan):
        idx, side = plan.quantize(c.contiguous(), steps)
        return plan.dequantize(idx, steps, side)

    @staticmethod
    def backward(ctx, g):
        return g, None, None


def ct_forward(x, plan):
    return CTForward.apply(x, plan)


def ct_inverse(c, plan):
    return CTInverse.apply(c, plan)


def st_quant(c, steps, plan):
    return STQuant.apply(c, steps, plan)


def rd_loss(c, x, steps, plan, lam):
    """||S Q_ST(c) - x||^2 + lam * ||c||_1, summed over the batch."""
    rec = ct_inverse(st_quant(c, steps, plan), plan)
    return ((rec - x) ** 2).sum() + lam * c.abs().sum()


def make_plan(height, width, levels, dirs, batch, device="cuda", filters="97", recon="dual"):
    """Plan for the functions above; filters and recon select the variants
    (see ct.geom): the adjoints follow the plan's filter pair and
    reconstruction."""
    return _ct.Plan(height, width, levels, dirs, batch, device, filters=filters, recon=recon)
