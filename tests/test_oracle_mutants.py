"""The oracle's pins catch plausible mistakes.

An independent numpy evaluation of the same definition is run through the
pin checks twice: as written (it must pass every check, like the oracle)
and with one planted mistake at a time (each must fail at least one check).
This shows the pins would notice such a mistake in the oracle itself.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]


def stored(buf, rows, cols, ld, dtype=np.float64):
    """rows x cols view of a column-major buffer at leading dimension ld."""
    if not rows or not cols:
        return np.zeros((rows, cols), dtype)
    buf = np.ascontiguousarray(buf)
    view = np.lib.stride_tricks.as_strided(buf, shape=(rows, cols),
                                           strides=(buf.itemsize, buf.itemsize * ld))
    return np.array(view, dtype=dtype)


def np_gemm(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc, bug=None):
    """C = alpha op(A) op(B) + beta C0 with numpy, optionally with a bug."""
    dt = np.float32 if bug == "f32_accumulate" else np.float64
    ra, ca = synth.stored_shape(transA, M, K)
    rb, cb = synth.stored_shape(transB, K, N)
    if bug == "ignore_lda":
        lda = max(1, ra)
    Asto = stored(A, ra, ca, lda, dt) if K and alpha != 0 else np.zeros((ra, ca), dt)
    Bsto = stored(B, rb, cb, ldb, dt) if K and alpha != 0 else np.zeros((rb, cb), dt)
    opA = Asto.T if transA in "TtCc" else Asto
    opB = Bsto.T if transB in "TtCc" else Bsto
    if bug == "transpose_a" and opA.shape[0] == opA.shape[1]:
        opA = opA.T
    if bug == "skip_last_k" and K > 0:
        opA, opB = opA[:, :-1], opB[:-1, :]
    a = -alpha if bug == "alpha_sign" else alpha
    prod = np.zeros((M, N), dt)
    if K and alpha != 0:
        if dt == np.float32:            # sequential FP32 accumulation
            for k in range(opA.shape[1]):
                prod = (prod + np.outer(opA[:, k], opB[k, :]).astype(np.float32)).astype(np.float32)
        else:
            prod = opA @ opB
    out = a * prod.astype(np.float64)
    if bug == "drop_beta":
        return out
    if beta != 0 or (bug == "reads_c_when_beta_zero" and C0 is not None):
        out = out + beta * stored(C0, M, N, ldc)
    return out


# ---- pin checks, parametrised by the implementation under test ----------------

def brute_force_ok(gemm):
    for ta, tb in TRANS:
        for (M, N, K) in ((3, 5, 4), (7, 2, 8), (5, 6, 1), (4, 3, 4)):
            c = synth.sgemm_case(11 + M * 100 + N * 10 + K, ta, tb, M, N, K, alpha=-1.25,
                                 beta=0.75, pad=3)
            got = gemm(ta, tb, M, N, K, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                       c["beta"], c["C"], c["ldc"])
            opA = stored(c["A"], *synth.stored_shape(ta, M, K), c["lda"])
            opA = opA.T if ta == "T" else opA
            opB = stored(c["B"], *synth.stored_shape(tb, K, N), c["ldb"])
            opB = opB.T if tb == "T" else opB
            C0 = stored(c["C"], M, N, c["ldc"])
            if not np.all(np.isfinite(got)):   # NaN padding reached the result
                return False
            for i in range(M):
                for j in range(N):
                    s = sum((Fraction(opA[i, k]) * Fraction(opB[k, j]) for k in range(K)),
                            Fraction(0))
                    exact = Fraction(float(c["alpha"])) * s + Fraction(float(c["beta"])) * \
                        Fraction(C0[i, j])
                    mag = 1.25 * float(np.sum(np.abs(opA[i, :] * opB[:, j]))) + 0.75 * abs(C0[i, j])
                    if abs(Fraction(float(got[i, j])) - exact) > (K + 2) * 2.0 ** -53 * mag + 1e-300:
                        return False
    return True


def beta_zero_ok(gemm):
    c = synth.sgemm_case(2, "N", "N", 8, 8, 8)
    C0 = np.full_like(c["C"], np.nan)
    got = gemm("N", "N", 8, 8, 8, 1.0, c["A"], c["lda"], c["B"], c["ldb"], 0.0, C0, c["ldc"])
    return bool(np.all(np.isfinite(got)))


def row_sum_ok(gemm):
    M, N, K = 23, 3, 301
    rng = np.random.default_rng(8)
    A = synth.matrix(rng, M, K, M + 5)
    B = np.ones(K * N, dtype=np.float32)
    got = gemm("N", "N", M, N, K, 0.5, A, M + 5, B, K, 0.0, None, M)
    opA = stored(A, M, K, M + 5)
    for i in range(M):
        want = 0.5 * math.fsum(opA[i])
        if abs(got[i, 0] - want) > K * 2.0 ** -53 * float(np.sum(np.abs(opA[i]))):
            return False
    return True


CHECKS = [brute_force_ok, beta_zero_ok, row_sum_ok]
BUGS = ["drop_beta", "alpha_sign", "ignore_lda", "skip_last_k", "transpose_a",
        "f32_accumulate", "reads_c_when_beta_zero"]


def test_the_oracle_passes_every_check():
    for check in CHECKS:
        assert check(oracle.sgemm), check.__name__


def test_the_clean_numpy_evaluation_passes_every_check():
    for check in CHECKS:
        assert check(np_gemm), check.__name__


@pytest.mark.parametrize("bug", BUGS)
def test_each_planted_mistake_is_caught(bug):
    def mutant(*args):
        return np_gemm(*args, bug=bug)
    failed = [check.__name__ for check in CHECKS if not check(mutant)]
    assert failed, "no pin catches %s" % bug
