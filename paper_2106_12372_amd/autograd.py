"""torch.autograd.Function over the fused HIP forward and backward kernels.

The weights are an ordinary FP32 device tensor (a torch Parameter), so any
torch optimiser can drive them; each forward and backward call uploads them
into the cache (a device-to-device copy plus the rebuild of the FP16/BF16
operand copies).  By default the forward pass keeps every hidden layer's
activations in a buffer (nrc_forward_train) that the backward pass reads
(Sec. 4, "Training the fully fused neural network"); with
keep_activations=False the backward kernel recomputes them instead, trading
the buffer (n x hidden x width values) for a second forward pass.
"""
from __future__ import annotations

import numpy as np
import torch

import synthdata as sd
from . import nrc as N


class NRCFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, enc, weights, cache, keep_activations=True):
        w = weights.detach().contiguous()
        cache.set_weights_device(w)
        enc_c = enc.detach().to(cache.enc_dtype).contiguous()
        if keep_activations:
            rgb, act = N.nrc_forward_train(cache, enc_c)
        else:
            rgb, act = N.nrc_forward(cache, enc_c), None
        ctx.save_for_backward(enc_c, w)
        ctx.act = act
        ctx.cache = cache
        ctx.enc_dtype = enc.dtype
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        enc_c, w = ctx.saved_tensors
        cache = ctx.cache
        cache.set_weights_device(w)
        grad_w, grad_enc = N.nrc_backward(cache, enc_c, grad_rgb.detach().float().contiguous(),
                                          want_grad_enc=ctx.needs_input_grad[0], act=ctx.act)
        ctx.act = None
        if grad_enc is not None:
            grad_enc = grad_enc.to(ctx.enc_dtype)
        return grad_enc, grad_w, None, None


class NRCModule(torch.nn.Module):
    """The cache network as a torch module: weights are one flat Parameter."""

    def __init__(self, width: int = 64, n_hidden: int = 5, precision: str = "fp16",
                 weights: np.ndarray | None = None, device=None, keep_activations: bool = True, **config):
        """config: further nrc_config fields (enc_preset, factorize, ...)."""
        super().__init__()
        self.keep_activations = keep_activations
        self.cache = N.Cache(N.make_config(width=width, n_hidden=n_hidden, precision=precision, **config),
                             device=device)
        w = sd.glorot_weights(width, n_hidden) if weights is None else np.asarray(weights, np.float32)
        self.weights = torch.nn.Parameter(torch.from_numpy(w.copy()).to(self.cache.device))

    def forward(self, enc):
        return NRCFunction.apply(enc, self.weights, self.cache, self.keep_activations)
