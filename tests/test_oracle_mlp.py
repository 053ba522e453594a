"""Pins of the FP64 multilayer-perceptron oracle (the application of the
paper's Section 4: a neural network trained with SGEMM as its kernel).

The pins do not retype the oracle's formulas:
* hand-worked one-unit networks, whose loss and gradients are written down
  as numbers;
* central finite differences of the loss, against the backpropagated
  gradients, on a small three-layer network (widths 4, 6, 6, 3: one square
  layer, so a weight used untransposed still has the right shape);
* the step goes downhill for a small learning rate.
A numpy copy of the same definition with one planted mistake at a time must
fail at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def hand_cases():
    """(Ws, X, T, loss, [dW_l]) worked by hand."""
    out = []
    # One linear layer, B = 2: H = X W = [0.5, 1]; loss = 0.5/2 (0.25 + 1).
    # dW = X^T (H - T) / B = (1*0.5 + 2*1) / 2 = 1.25.
    out.append(([np.array([[0.5]])], np.array([[1.0], [2.0]]), np.array([[0.0], [0.0]]),
                0.3125, [np.array([[1.25]])]))
    # tanh hidden unit then a linear output, B = 1: W1 = atanh(0.5) so
    # H1 = 0.5, W2 = 2 so H2 = 1, T = 0: loss 0.5; dW2 = H1 * 1 = 0.5;
    # G1 = 1 * W2 * (1 - 0.25) = 1.5, dW1 = X * G1 = 1.5.
    out.append(([np.array([[math.atanh(0.5)]]), np.array([[2.0]])], np.array([[1.0]]),
                np.array([[0.0]]), 0.5, [np.array([[1.5]]), np.array([[0.5]])]))
    return out


def fd_case():
    X, T, Ws = synth.mlp_case(3, 5, [4, 6, 6, 3])
    return [W.astype(np.float64) for W in Ws], X.astype(np.float64), T.astype(np.float64)


def check_hand(loss_fn, grads_fn):
    for Ws, X, T, loss, dWs in hand_cases():
        if not math.isclose(loss_fn(Ws, X, T), loss, rel_tol=1e-12):
            return False
        _, g = grads_fn(Ws, X, T)
        if any(not np.allclose(a, b, rtol=1e-12, atol=0) for a, b in zip(g, dWs)):
            return False
    return True


def check_fd(loss_fn, grads_fn, h=1e-6):
    Ws, X, T = fd_case()
    _, g = grads_fn(Ws, X, T)
    scale = max(float(np.max(np.abs(d))) for d in g)
    rng = np.random.default_rng(0)
    for l, W in enumerate(Ws):
        for _ in range(6):
            i, j = rng.integers(0, W.shape[0]), rng.integers(0, W.shape[1])
            up = [w.copy() for w in Ws]
            dn = [w.copy() for w in Ws]
            up[l][i, j] += h
            dn[l][i, j] -= h
            fd = (loss_fn(up, X, T) - loss_fn(dn, X, T)) / (2 * h)
            if abs(fd - g[l][i, j]) > 1e-7 * scale:
                return False
    return True


def check_descent(loss_fn, step_fn):
    Ws, X, T = fd_case()
    before = loss_fn(Ws, X, T)
    _, new = step_fn(Ws, X, T, 1e-2)
    return loss_fn(new, X, T) < before


def test_oracle_hand_worked_networks():
    assert check_hand(oracle.mlp_loss, oracle.mlp_grads)


def test_oracle_gradients_match_finite_differences():
    assert check_fd(oracle.mlp_loss, oracle.mlp_grads)


def test_oracle_step_goes_downhill():
    assert check_descent(oracle.mlp_loss, oracle.mlp_step)


def test_oracle_loss_returned_with_gradients():
    Ws, X, T = fd_case()
    loss, _ = oracle.mlp_grads(Ws, X, T)
    assert loss == oracle.mlp_loss(Ws, X, T)


# --- planted mistakes --------------------------------------------------------
BUGS = [None, "no_tanh_derivative", "grad_not_divided_by_batch", "loss_and_grad_not_divided",
        "tanh_on_output", "w_not_transposed", "step_uphill", "derivative_from_next_layer"]


def np_mlp(bug):
    """(loss_fn, grads_fn, step_fn) of a numpy copy with one planted bug."""
    def forward(Ws, X):
        H = [X]
        for l, W in enumerate(Ws):
            Z = H[-1] @ W
            top = l + 1 == len(Ws)
            H.append(np.tanh(Z) if (not top or bug == "tanh_on_output") else Z)
        return H

    def loss_fn(Ws, X, T):
        E = forward(Ws, X)[-1] - T
        s = 0.5 * float(np.sum(E * E))
        return s if bug == "loss_and_grad_not_divided" else s / E.shape[0]

    def grads_fn(Ws, X, T):
        H = forward(Ws, X)
        E = H[-1] - T
        B = E.shape[0]
        G = E if bug in ("grad_not_divided_by_batch", "loss_and_grad_not_divided") else E / B
        if bug == "tanh_on_output":
            pass            # the forward is wrong; the backward is left as written
        dWs = [None] * len(Ws)
        for l in range(len(Ws) - 1, -1, -1):
            dWs[l] = H[l].T @ G
            if l > 0:
                Wl = Ws[l]
                back = G @ (Wl if (bug == "w_not_transposed" and Wl.shape[0] == Wl.shape[1]) else Wl.T)
                Hd = H[l + 1] if bug == "derivative_from_next_layer" and H[l + 1].shape == H[l].shape else H[l]
                G = back if bug == "no_tanh_derivative" else back * (1.0 - Hd * Hd)
        return loss_fn(Ws, X, T), dWs

    def step_fn(Ws, X, T, lr):
        loss, dWs = grads_fn(Ws, X, T)
        sgn = -1.0 if bug == "step_uphill" else 1.0
        return loss, [W - sgn * lr * d for W, d in zip(Ws, dWs)]
    return loss_fn, grads_fn, step_fn


@pytest.mark.parametrize("bug", BUGS)
def test_pins_catch_planted_mistakes(bug):
    loss_fn, grads_fn, step_fn = np_mlp(bug)
    ok = (check_hand(loss_fn, grads_fn) and check_fd(loss_fn, grads_fn)
          and check_descent(loss_fn, step_fn))
    assert ok == (bug is None), bug
