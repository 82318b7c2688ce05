"""torch.autograd.Function around the hand-written forward/backward kernels.

``render(params, model, view, pix, jitter)`` returns the ray sums A (Eq. 1) of the given rays as a
differentiable function of the model's flat parameter tensor: the forward pass runs ``nic_forward``,
the backward pass runs ``nic_backward`` with the upstream gradient dL/dA and returns the gradient
of every parameter (table, LayerNorm, MLP) as one flat tensor.  Any loss written in torch on top of
A (for example Eq. 3's L1) can then be optimised with the library's Adam or a torch optimiser.
"""
from __future__ import annotations

import torch


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, model, view, pix, jitter):
        ctx.model = model
        ctx.view = int(view)
        ctx.save_for_backward(pix, jitter)
        return model.forward(ctx.view, pix, jitter)

    @staticmethod
    def backward(ctx, dA):
        pix, jitter = ctx.saved_tensors
        m = ctx.model
        m.zero_grad()
        m.backward(ctx.view, pix, jitter, dA.detach().to(torch.float32).contiguous())
        return m.tensors()[1].clone(), None, None, None, None


def leaf_params(model):
    """The model's FP32 parameter vector as a leaf tensor that requires grad (shares storage)."""
    p = model.tensors()[0]
    p.requires_grad_(True)
    return p


def render(params, model, view, pix, jitter):
    return _Render.apply(params, model, view, pix, jitter)
