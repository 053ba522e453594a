"""Multilayer-perceptron training steps on the library (the application of
the paper's Section 4) against the FP64 oracle.

Tolerances, normwise relative (Frobenius):
* FP32: each product of depth K <= 8192 errs by about sqrt(K) u times its
  absolute product, at most about 1e-6 here; tanh and the elementwise steps
  add a few u; the three layers of forward and backward chain about six
  such errors: 1e-5 leaves a margin of about 10.
* BF16x3: each product errs by about 4e-6 (the split's dropped lo*lo term
  and the bf16 rounding of lo); six in a chain: 5e-5.
The fused update W - lr dW is compared on the change lr dW (whose own
rounding, u |W|, is far below these bounds at the learning rates used).
"""
import numpy as np
import pytest

import oracle
import synth
import paper_1912_04379_amd as mg
from gpu_util import log

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 5e-5}
SMALL = (200, [96, 130, 70, 33])   # several tiles in every product, ragged edges


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make(seed, batch, widths, prec):
    X, T, Ws = synth.mlp_case(seed, batch, widths)
    net = mg.MLP([to_dev(W) for W in Ws], precision=prec)
    return X, T, Ws, net


def rel(a, b):
    return oracle.normwise_rel_err(np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_gradients_match_oracle(prec):
    batch, widths = SMALL
    X, T, Ws, net = make(11, batch, widths, prec)
    log("mlp grads %s batch %d widths %s" % (prec, batch, widths))
    loss, dWs = net.grads(to_dev(X), to_dev(T))
    ref_loss, ref = oracle.mlp_grads(Ws, X, T)
    assert abs(float(loss) - ref_loss) <= TOL[prec] * ref_loss
    for l, (d, r) in enumerate(zip(dWs, ref)):
        e = rel(d.cpu().numpy(), r)
        log("  layer %d: normwise rel err %.2e" % (l + 1, e))
        assert e <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_step_matches_oracle(prec):
    """The update fused into the weight-gradient products (alpha = -lr,
    beta = 1, C = W): the new weights against the oracle's, measured on
    the change of each weight matrix."""
    batch, widths = SMALL
    lr = 0.5
    X, T, Ws, net = make(12, batch, widths, prec)
    log("mlp step %s lr %g" % (prec, lr))
    loss = net.step(to_dev(X), to_dev(T), lr)
    ref_loss, ref_new = oracle.mlp_step(Ws, X, T, lr)
    assert abs(float(loss) - ref_loss) <= TOL[prec] * ref_loss
    for l, (W, Wold, Wref) in enumerate(zip(net.weights, Ws, ref_new)):
        change = Wref - Wold.astype(np.float64)
        e = np.linalg.norm(W.cpu().numpy().astype(np.float64) - Wref) / np.linalg.norm(change)
        log("  layer %d: error / change %.2e" % (l + 1, e))
        assert e <= TOL[prec]


def test_training_lowers_the_loss():
    """Ten steps of gradient descent on one batch: the loss falls at every
    step, and the last loss matches the oracle's after the same ten steps."""
    batch, widths = SMALL
    X, T, Ws, net = make(13, batch, widths, "fp32")
    Xd, Td = to_dev(X), to_dev(T)
    losses = [float(net.step(Xd, Td, 0.2)) for _ in range(10)]
    log("mlp losses " + " ".join("%.5f" % v for v in losses))
    assert all(b < a for a, b in zip(losses, losses[1:]))
    ref = [w.astype(np.float64) for w in Ws]
    for _ in range(9):
        _, ref = oracle.mlp_step(ref, X, T, 0.2)
    assert abs(losses[-1] - oracle.mlp_loss(ref, X, T)) <= 1e-4 * losses[-1]


def test_bench_shape_gradients():
    """The benchmark's network (batch 8192, widths 1024, 4096, 4096, 1024)
    at full size: every weight gradient of both FP32-accurate forms against
    the oracle (about 1.2e12 FP64 flops on the host)."""
    batch, widths = 8192, [1024, 4096, 4096, 1024]
    X, T, Ws = synth.mlp_case(0, batch, widths)
    ref_loss, ref = oracle.mlp_grads(Ws, X, T)
    for prec in ("fp32", "bf16x3"):
        net = mg.MLP([to_dev(W) for W in Ws], precision=prec)
        loss, dWs = net.grads(to_dev(X), to_dev(T))
        log("mlp bench shape %s: loss %.6f (oracle %.6f)" % (prec, float(loss), ref_loss))
        assert abs(float(loss) - ref_loss) <= TOL[prec] * ref_loss
        for l, (d, r) in enumerate(zip(dWs, ref)):
            e = rel(d.cpu().numpy(), r)
            log("  layer %d: normwise rel err %.2e" % (l + 1, e))
            assert e <= TOL[prec]
