"""Multilayer-perceptron training on the library's products.

The paper's application (Section 4) is the distributed training of a large
neural network with this SGEMM as the kernel of the training procedure.  The
paper names no architecture, loss or update rule; the network here is the
plain reading of it:

    H_0 = X (B x n_0),   H_l = tanh(H_{l-1} W_l) for hidden layers,
    H_L = H_{L-1} W_L (linear output),   loss = 0.5 / B * ||H_L - T||_F^2,

and one step of gradient descent, W_l <- W_l - lr dL/dW_l, by
backpropagation:

    G_L = (H_L - T) / B
    dL/dW_l = H_{l-1}^T G_l
    G_{l-1} = (G_l W_l^T) o (1 - H_{l-1}^2)        (l > 1)

Every product is one library call on row-major tensors, and the
elementwise work around the products is fused into their epilogues:
* the hidden layers' tanh into the forward products (the library's tanh
  activation), so each H_l is stored once, already activated;
* the tanh derivative into the input-gradient products (the tanh_grad
  activation with aux = H_{l-1}): G_{l-1} = (G_l W_l^T) o (1 - H_{l-1}^2) in
  one pass;
* the update into the weight-gradient product: C = W_l, alpha = -lr, beta =
  1 computes W_l - lr H_{l-1}^T G_l, so the gradient is never stored and the
  weights are read and written once.  G_{l-1} is formed from W_l before that
  update.
Only the output error (H_L - T) / B and the loss are torch operations.
"""
import torch

from .api import matmul


def step_flops(batch, widths):
    """Flops of the products of one training step: the forward products,
    the input-gradient products of layers 2..L and the weight-gradient
    products, 2 per multiply-add."""
    layers = list(zip(widths[:-1], widths[1:]))
    fwd = sum(2 * batch * a * b for a, b in layers)
    dx = sum(2 * batch * a * b for a, b in layers[1:])
    return fwd + dx + fwd


class MLP:
    """Weights W_1..W_L: float32 contiguous (n_{l-1} x n_l) device tensors,
    updated in place by ``step``.  ``precision`` selects the products' form
    ("fp32" or "bf16x3"; "fp16s" also runs but is not FP32-accurate)."""

    def __init__(self, weights, precision="fp32"):
        if not weights:
            raise ValueError("at least one layer")
        for a, b in zip(weights[:-1], weights[1:]):
            if a.shape[1] != b.shape[0]:
                raise ValueError("layer widths do not chain: %s then %s"
                                 % (tuple(a.shape), tuple(b.shape)))
        for W in weights:
            if W.dtype != torch.float32 or not W.is_contiguous() or W.dim() != 2:
                raise ValueError("weights must be contiguous 2-D float32 tensors")
        self.weights = list(weights)
        self.precision = precision

    def forward(self, X):
        """[H_0 = X, H_1, ..., H_L]."""
        H = [X]
        last = len(self.weights) - 1
        for l, W in enumerate(self.weights):
            H.append(matmul(H[-1], W, precision=self.precision,
                            activation="tanh" if l < last else None))
        return H

    def _output_gradient(self, H, T):
        """(loss as a 0-d device tensor, G_L = (H_L - T) / B)."""
        B = H[-1].shape[0]
        G = H[-1] - T
        loss = G.pow(2).sum() * (0.5 / B)
        G.mul_(1.0 / B)
        return loss, G

    def grads(self, X, T):
        """(loss, [dL/dW_l]) without changing the weights."""
        H = self.forward(X)
        loss, G = self._output_gradient(H, T)
        dWs = [None] * len(self.weights)
        for l in range(len(self.weights) - 1, -1, -1):
            dWs[l] = matmul(H[l].t(), G, precision=self.precision)
            if l > 0:
                G = self._backward_input(G, l, H)
        return loss, dWs

    def _backward_input(self, G, l, H):
        # (G W_l^T) o (1 - H_{l-1}^2) in one library call: the product with
        # the tanh derivative in its epilogue (H[l] is H_{l-1}).
        return matmul(G, self.weights[l].t(), precision=self.precision,
                      activation="tanh_grad", aux=H[l])

    def step(self, X, T, lr):
        """One gradient-descent step on the batch (X, T); returns the loss
        before the step as a 0-d device tensor (no synchronisation)."""
        H = self.forward(X)
        loss, G = self._output_gradient(H, T)
        for l in range(len(self.weights) - 1, -1, -1):
            Gp = self._backward_input(G, l, H) if l > 0 else None
            W = self.weights[l]
            matmul(H[l].t(), G, alpha=-lr, beta=1.0, out=W, precision=self.precision)
            G = Gp
        return loss
