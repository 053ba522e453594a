"""mgemm_sgemm_act: an activation fused into the product's epilogue.

C <- tanh(v) or C <- v (1 - aux^2), with v = alpha op(A) op(B) + beta C.
The reference is the oracle's FP64 product v with the activation applied in
FP64.  tanh is 1-Lipschitz and |1 - y^2| <= 1 for |y| <= 1, so the
activated result errs by at most the product's own error plus the
rounding of the activation itself (a few units in the last place of the
result).  The bars are therefore the product's: normwise, ||got - ref|| <=
tol ||v|| + 8u ||ref|| (the activation shrinks the result's norm more than
its error, so a bar relative to ||ref|| would not follow from the
product's); elementwise (FP32), the product's gamma bound times the
activation's slope plus 4 ulp of the result.
"""
import os

import numpy as np
import pytest

import oracle
import paper_1912_04379_amd as mg
import synth
from gpu_util import fp32_bound, log, logical_c, oracle_args, padding_untouched, to_dev
from paper_1912_04379_amd import _lib

U = 2.0 ** -24


def _aux(case, seed):
    """An M x N array at C's leading dimension, values of tanh's range."""
    rng = np.random.default_rng(seed)
    a = synth.matrix(rng, case["M"], case["N"], case["ldc"], pad=np.float32(0.0))
    return np.tanh(a.astype(np.float64) * 1.5).astype(np.float32)


def _run(case, prec, cfg, act, aux):
    import torch
    A, B, C = to_dev(case["A"]), to_dev(case["B"]), to_dev(case["C"])
    X = to_dev(aux) if aux is not None else None
    mg.sgemm(case["transA"], case["transB"], case["M"], case["N"], case["K"],
             float(case["alpha"]), A, case["lda"], B, case["ldb"], float(case["beta"]), C,
             case["ldc"], precision=prec, config=cfg, activation=act, aux=X)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:case["C"].size]


def _check(case, prec, got_buf, act, aux, normwise):
    v = oracle.sgemm(*oracle_args(case))
    got = logical_c(got_buf, case)
    assert padding_untouched(got_buf, case), "C padding was written"
    if act == "tanh":
        ref = np.tanh(v)
        lip = np.ones_like(v)
    else:
        y = aux.reshape(case["N"], case["ldc"])[:, :case["M"]].T.astype(np.float64)
        lip = 1.0 - y * y
        ref = v * lip
    err = np.linalg.norm(got - ref) / max(np.linalg.norm(v), 1e-300)
    bar = normwise + 8 * U * np.linalg.norm(ref) / max(np.linalg.norm(v), 1e-300)
    assert err <= bar, "%s %s: ||got - ref|| / ||v|| = %.3e > %.3e" % (prec, act, err, bar)
    if prec == "fp32":
        bound = fp32_bound(case) * np.abs(lip) + 4 * U * np.abs(ref) + 1e-30
        bad = np.abs(got - ref) > bound
        assert not bad.any(), "elementwise bound violated at %s" % (np.argwhere(bad)[:4],)
    return err


CASES = [
    # precision, configuration, shape, trans
    ("fp32", -1, (300, 260, 700), "NT"),
    ("fp32", 0, (257, 255, 33), "TN"),
    ("fp32", 9, (100, 90, 500), "NN"),        # the small-product kernel
    ("fp32", 10, (600, 520, 4200), "TT"),     # 256 x 256 rounds with a 128 x 128 tail
    ("fp32", 11, (200, 136, 5000), "NN"),     # split-K: the activation in the reduction
    ("bf16x3", -1, (300, 260, 700), "NT"),
    ("bf16x3", 0, (520, 390, 200), "TN"),
    ("bf16x3", 11, (520, 390, 600), "NN"),    # packed
    ("bf16x3", 13, (200, 136, 5000), "TT"),   # split-K
    ("fp16s", -1, (300, 260, 700), "NN"),
    ("fp16s", 12, (520, 390, 3100), "TN"),    # packed, 32-deep stages
    ("fp16s", 13, (200, 136, 5000), "NT"),    # split-K
]


@pytest.mark.gpu
@pytest.mark.parametrize("act", ["tanh", "tanh_grad"])
@pytest.mark.parametrize("prec,cfg,shape,trans", CASES)
def test_fused_activation_against_the_oracle(prec, cfg, shape, trans, act):
    M, N, K = shape
    c = synth.sgemm_case(41, trans[0], trans[1], M, N, K, alpha=0.7, beta=-0.5, pad=3)
    aux = _aux(c, 42) if act == "tanh_grad" else None
    log("%s cfg %d %s %s %s" % (prec, cfg, shape, trans, act))
    got = _run(c, prec, cfg, act, aux)
    _check(c, prec, got, act, aux, 1e-3 if prec == "fp16s" else 1e-5)


@pytest.mark.gpu
@pytest.mark.parametrize("act", ["tanh", "tanh_grad"])
def test_fused_activation_without_a_product(act):
    """alpha = 0 (and K = 0): C <- act(beta C); with beta = 1 the quick
    return does not apply, C <- act(C)."""
    for alpha, K, beta in ((0.0, 40, 1.0), (1.0, 0, 1.0), (0.0, 40, -2.0)):
        c = synth.sgemm_case(43, "N", "N", 70, 33, K, alpha=alpha, beta=beta, pad=2)
        aux = _aux(c, 44) if act == "tanh_grad" else None
        log("no product: alpha %g K %d beta %g %s" % (alpha, K, beta, act))
        got = _run(c, "fp32", -1, act, aux)
        _check(c, "fp32", got, act, aux, 1e-6)


@pytest.mark.gpu
def test_fused_activation_on_the_64_bit_address_path():
    """ldc beyond the buffer path's limit: the 64-bit epilogue applies the
    activation too."""
    from gpu_util import wide_ldc_case
    c = wide_ldc_case(45, "N", "T", 130, 7, 90, alpha=1.5, beta=-0.5)
    for act in ("tanh", "tanh_grad"):
        aux = _aux(c, 46) if act == "tanh_grad" else None
        log("64-bit path %s" % act)
        got = _run(c, "fp32", -1, act, aux)
        _check(c, "fp32", got, act, aux, 1e-5)


@pytest.mark.gpu
def test_fused_tanh_matches_product_then_torch_tanh():
    """The fused call stores tanhf of the same FP32 value the plain call
    stores: torch's tanh of the plain result agrees within 2 ulp (the two
    tanh implementations may round differently)."""
    import torch
    c = synth.sgemm_case(47, "T", "N", 384, 320, 1024, alpha=1.0, beta=0.0, pad=0)
    A, B = to_dev(c["A"]), to_dev(c["B"])
    C1, C2 = to_dev(c["C"]), to_dev(c["C"])
    for prec in ("fp32", "bf16x3"):
        mg.sgemm("T", "N", 384, 320, 1024, 1.0, A, c["lda"], B, c["ldb"], 0.0, C1, c["ldc"],
                 precision=prec)
        mg.sgemm("T", "N", 384, 320, 1024, 1.0, A, c["lda"], B, c["ldb"], 0.0, C2, c["ldc"],
                 precision=prec, activation="tanh")
        torch.cuda.synchronize()
        d = (torch.tanh(C1) - C2).abs() / C2.abs().clamp_min(1e-30)
        assert float(d.max()) <= 2.0 ** -22, prec


# ---- argument checks (no device work) ----------------------------------------

FA, FB, FC, FX = 0x10000000, 0x20000000, 0x30000000, 0x40000000


def _act(activation, aux=FX, C=FC, **kw):
    a = dict(transA=b"N", transB=b"N", M=4, N=4, K=4, alpha=1.0, A=FA, lda=4, B=FB, ldb=4,
             beta=0.0, C=C, ldc=4)
    a.update(kw)
    return mg.lib().mgemm_sgemm_act(a["transA"], a["transB"], a["M"], a["N"], a["K"],
                                    a["alpha"], a["A"], a["lda"], a["B"], a["ldb"], a["beta"],
                                    a["C"], a["ldc"], None, 0, -1, activation, aux)


def test_activation_argument_errors():
    assert _act(7) == _lib.ERR_UNSUPPORTED
    assert b"activation" in mg.lib().mgemm_last_error()
    assert _act(2, aux=None) == _lib.ERR_UNSUPPORTED
    assert b"aux" in mg.lib().mgemm_last_error()
    assert _act(2, aux=FC + 8) == _lib.ERR_ALIAS
    assert b"aux" in mg.lib().mgemm_last_error()
    # BLAS argument errors keep their numbers and come first.
    assert _act(9, lda=3) == -8
    # M = 0: nothing to do, whatever the activation.
    assert _act(2, aux=None, M=0, C=None) == 0


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="would reach a launch on a GPU")
def test_activation_disables_the_quick_return():
    """alpha = 0, beta = 1 returns at once without an activation; with one,
    C <- act(C) must run, so the call goes on to the device check."""
    assert _act(0, alpha=0.0, beta=1.0) == 0
    assert _act(1, alpha=0.0, beta=1.0) == _lib.ERR_NO_DEVICE
