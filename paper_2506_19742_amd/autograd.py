"""torch.autograd.Function around the hand-written forward/backward kernels.

``render(params, model, view, pix, jitter)`` returns the ray sums A (Eq. 1) of the given rays as a
differentiable function of the model's flat parameter tensor: the forward pass runs ``nic_forward``,
the backward pass runs ``nic_backward`` with the upstream gradient dL/dA and returns the gradient
of every parameter (table, LayerNorm, MLP) as one flat tensor.  Any loss written in torch on top of
A (for example Eq. 3's L1) can then be optimised with the library's Adam or a torch optimiser.

``params`` must be the model's own parameter storage (``leaf_params``): the kernels read the
parameters from the model, so a different tensor is refused.  The backward pass hands torch a copy
of the gradient and leaves the library's gradient buffer at zero, so a later ``nic_step`` does not
apply it a second time.  In the precision form (FP16 table copy for the gathers) the forward pass
refreshes that copy from the FP32 parameters first, so torch-side updates are always seen.
"""
from __future__ import annotations

import torch


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, model, view, pix, jitter):
        own = model.tensors()[0]
        if params.data_ptr() != own.data_ptr() or params.numel() != own.numel():
            raise ValueError("params must be the model's parameter tensor (autograd.leaf_params(model))")
        if model.cfg.precision:
            model.sync_params()          # FP16 table copy from the (possibly torch-updated) FP32 table
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
        g = m.tensors()[1].clone()
        m.zero_grad()                    # nothing stays pending for the library's own Adam
        return g, None, None, None, None


def leaf_params(model):
    """The model's FP32 parameter vector as a leaf tensor that requires grad (shares storage)."""
    p = model.tensors()[0]
    p.requires_grad_(True)
    return p


def render(params, model, view, pix, jitter):
    return _Render.apply(params, model, view, pix, jitter)
