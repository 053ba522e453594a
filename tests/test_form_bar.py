"""The statistical bar of tests/form_bars.py is tight enough to catch the
mistakes it is meant for, and loose enough for correct FP32 accumulation.

A numpy model of the kernels' accumulation is run on the CPU: the form's
terms in blocks of 16 k (one MFMA), each block's exact sum added to an FP32
accumulator with one rounding, the three products of the split form in
turn, then the FP32 epilogue fma(beta, C, alpha*acc).  Run faithfully, it
stays well inside the bar; with a planted mistake (a truncating split, a
dropped correction term, a kept lo*lo, a truncating FP16 conversion) it
exceeds the bar on the same inputs.
"""
import numpy as np
import pytest

import oracle
import synth
from form_bars import stat_bar


def _rz_bf16(x):
    return (np.asarray(x, np.float32).view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)


def _rz_f16(x):
    x = np.asarray(x, np.float64)
    h = x.astype(np.float16)
    over = np.abs(h.astype(np.float64)) > np.abs(x)
    return np.where(over, np.nextafter(h, np.float16(0)), h).astype(np.float64)


def _accumulate(pairs, K, M, N):
    acc = np.zeros((M, N), np.float32)
    for k0 in range(0, K, 16):
        for a, b in pairs:
            s = a[:, k0:k0 + 16] @ b[k0:k0 + 16]
            acc = (acc.astype(np.float64) + s).astype(np.float32)
    return acc


def _epilogue(c, acc):
    C0 = c["C"].reshape(c["N"], c["ldc"])[:, :c["M"]].T.astype(np.float64)
    t = (np.float32(c["alpha"]) * acc).astype(np.float32).astype(np.float64)
    return (np.float64(c["beta"]) * C0 + t).astype(np.float32).astype(np.float64)


def model_bf16x3(c, bug=None):
    M, N, K = c["M"], c["N"], c["K"]
    opA = oracle.op_matrix(c["A"], c["lda"], c["transA"], M, K)
    opB = oracle.op_matrix(c["B"], c["ldb"], c["transB"], K, N)
    if bug == "rz_split":
        split = lambda x: (_rz_bf16(x), _rz_bf16((x - _rz_bf16(x)).astype(np.float32)))
    else:
        split = oracle.split_bf16
    ah, al = (v.astype(np.float64) for v in split(opA))
    bh, bl = (v.astype(np.float64) for v in split(opB))
    pairs = [(ah, bh), (ah, bl), (al, bh)]
    if bug == "drop_lohi":
        pairs = pairs[:2]
    if bug == "keep_lolo":
        pairs.append((al, bl))
    return _epilogue(c, _accumulate(pairs, K, M, N))


def model_f16s(c, bug=None):
    M, N, K = c["M"], c["N"], c["K"]
    eA, eB = oracle.f16_exponents(c["transA"], c["transB"], M, N, K, c["A"], c["lda"],
                                  c["B"], c["ldb"])
    rA = np.repeat(eA, 32)[:M].astype(np.float64)
    cB = np.repeat(eB, 32)[:N].astype(np.float64)
    opA = oracle.op_matrix(c["A"], c["lda"], c["transA"], M, K).astype(np.float64)
    opB = oracle.op_matrix(c["B"], c["ldb"], c["transB"], K, N).astype(np.float64)
    conv = _rz_f16 if bug == "rz_f16" else (lambda x: x.astype(np.float16).astype(np.float64))
    qA = conv(opA * np.exp2(rA)[:, None])
    qB = conv(opB * np.exp2(cB)[None, :])
    acc = _accumulate([(qA, qB)], K, M, N)
    acc = (acc.astype(np.float64) * np.exp2(-(rA[:, None] + cB[None, :]))).astype(np.float32)
    return _epilogue(c, acc)


CASES = [(96, 80, 2048, "uniform"), (96, 80, 2048, "loguni"), (70, 90, 1000, "uniform"),
         (64, 64, 333, "loguni"), (33, 65, 77, "uniform"), (40, 24, 7, "uniform")]


def _case(M, N, K, dist):
    return synth.sgemm_case(61, "T", "N", M, N, K, alpha=1.5, beta=-0.5, pad=3, dist=dist)


def _ratio(c, got, emulate):
    a = (c["transA"], c["transB"], c["M"], c["N"], c["K"], c["alpha"], c["A"], c["lda"], c["B"],
         c["ldb"], c["beta"], c["C"], c["ldc"])
    return oracle.normwise_rel_err(got, emulate(*a)) / stat_bar(c["K"])


@pytest.mark.parametrize("M,N,K,dist", CASES)
def test_faithful_model_is_inside_the_bar(M, N, K, dist):
    c = _case(M, N, K, dist)
    assert _ratio(c, model_bf16x3(c), oracle.bf16x3) < 0.5
    assert _ratio(c, model_f16s(c), oracle.f16_scaled) < 0.5


@pytest.mark.parametrize("bug", ["rz_split", "drop_lohi", "keep_lolo"])
@pytest.mark.parametrize("M,N,K,dist", CASES)
def test_bf16x3_mistakes_exceed_the_bar(bug, M, N, K, dist):
    c = _case(M, N, K, dist)
    assert _ratio(c, model_bf16x3(c, bug), oracle.bf16x3) > 1.2


@pytest.mark.parametrize("M,N,K,dist", CASES)
def test_truncating_f16_conversion_exceeds_the_bar(M, N, K, dist):
    c = _case(M, N, K, dist)
    assert _ratio(c, model_f16s(c, "rz_f16"), oracle.f16_scaled) > 1.2
