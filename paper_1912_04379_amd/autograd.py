"""Dense layer Y = X W with a hand-written backward.

For L a scalar function of Y with G = dL/dY:
    dX = G W^T,   dW = X^T G.
Forward and backward are one library call each (row-major torch tensors
enter the column-major product through their storage; transposed views
become trans flags, so no copies are made).
"""
import torch

from .api import matmul


class MGemmLinear(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, W, precision="fp32"):
        ctx.save_for_backward(X, W)
        ctx.precision = precision
        return matmul(X, W, precision=precision)

    @staticmethod
    def backward(ctx, G):
        X, W = ctx.saved_tensors
        if G.stride(-1) != 1 and G.stride(0) != 1:
            G = G.contiguous()
        dX = dW = None
        if ctx.needs_input_grad[0]:
            dX = matmul(G, W.t(), precision=ctx.precision)     # G W^T
        if ctx.needs_input_grad[1]:
            dW = matmul(X.t(), G, precision=ctx.precision)     # X^T G
        return dX, dW, None


def linear(X, W, precision="fp32"):
    """Y = X @ W (float32 device tensors) with the library's backward."""
    return MGemmLinear.apply(X, W, precision)
