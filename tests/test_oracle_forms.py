"""Closed-form pins for the oracle's two emulated forms, and planted mistakes
they catch.

The split-precision form writes every FP32 value x as hi + lo, two BF16
values rounded to nearest (ties to even), and sums hi*hi + hi*lo + lo*hi;
the scaled FP16 form multiplies 32-row panels of op(A) and 32-column panels
of op(B), over the whole K, by powers of two chosen from each panel's
largest magnitude, rounds to FP16 and unscales exactly.  Neither is in the
paper; both are layered on the Section 1 product.

The expected values below are worked out by hand from IEEE rounding (the
derivation is written beside each constant), not computed by the oracle's
own code.  The same checks are run against an independent numpy evaluation,
as written (it must pass, like the oracle) and with one planted mistake at
a time (each must fail at least one check).
"""
import types
from fractions import Fraction

import numpy as np
import pytest

import oracle

F = Fraction
P = F(2)

# Hand-worked BF16 splits (7 fraction bits: spacing 2**-7 on [1, 2), 2**-6 on
# [2, 4), 2**-8 on [1/2, 1)).  Each entry: x, hi, lo.
SPLITS = [
    # 1 + 2^-8 + 2^-10 is 3*2^-10 below 1 + 2^-7 and 5*2^-10 above 1:
    # hi = 1 + 2^-7, lo = -3*2^-10 (1.5 * 2^-9, a BF16 value).
    (1 + P ** -8 + P ** -10, 1 + P ** -7, -3 * P ** -10),
    # 1 + 2^-9: 2^-9 is below half a spacing, so hi = 1, lo = 2^-9.
    (1 + P ** -9, F(1), P ** -9),
    # -(2 + 2^-6 + 2^-12): 2 + 2^-6 is a BF16 value; the rest is lo.
    (-(2 + P ** -6 + P ** -12), -(2 + P ** -6), -(P ** -12)),
    # 3/4 + 3*2^-10: 3*2^-10 is 3/4 of a spacing (2^-8), so hi rounds up to
    # 3/4 + 2^-8 and lo = 3*2^-10 - 2^-8 = -2^-10.
    (F(3, 4) + 3 * P ** -10, F(3, 4) + P ** -8, -(P ** -10)),
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7; even is 1: hi = 1, lo = 2^-8.
    (1 + P ** -8, F(1), P ** -8),
    # 1 + 2^-8 + 2^-10 + 2^-20: hi = 1 + 2^-7 as in the first entry; x - hi
    # = -(3*2^-10 - 2^-20) has spacing 2^-16 in BF16 ([2^-9, 2^-8)), so the
    # 2^-20 is lost: lo = -3*2^-10.
    (1 + P ** -8 + P ** -10 + P ** -20, 1 + P ** -7, -3 * P ** -10),
]


def _as_f32(v):
    f = np.float32(float(v))
    assert F(float(f)) == v, "constant is not an FP32 value"
    return f


def bf16x3_closed_form_ok(impl):
    """op(A) (3 x 4) and op(B) (4 x 2) built from the split table, every
    trans pair and alpha = 1, beta = 0.  The form's result is
    sum_k hi_a hi_b + hi_a lo_b + lo_a hi_b with the hand-derived halves;
    with K <= 4 these sums are exact in FP64, so the comparison is bitwise.
    Keeping lo*lo, truncating instead of rounding, or any other split
    changes at least one entry."""
    M, K, N = 3, 4, 2
    ia = [[0, 1, 2, 3], [4, 5, 0, 2], [3, 3, 1, 5]]       # op(A)[i][k] -> table index
    ib = [[5, 2], [0, 4], [3, 1], [2, 0]]                  # op(B)[k][j]
    want = np.empty((M, N))
    for i in range(M):
        for j in range(N):
            s = F(0)
            for k in range(K):
                _, ha, la = SPLITS[ia[i][k]]
                _, hb, lb = SPLITS[ib[k][j]]
                s += ha * hb + ha * lb + la * hb
            want[i, j] = float(s)
            assert F(want[i, j]) == s
    opA = np.array([[_as_f32(SPLITS[t][0]) for t in row] for row in ia], dtype=np.float32)
    opB = np.array([[_as_f32(SPLITS[t][0]) for t in row] for row in ib], dtype=np.float32)
    for ta in "NT":
        for tb in "NT":
            SA = opA.T if ta == "T" else opA
            SB = opB.T if tb == "T" else opB
            A = np.asfortranarray(SA).ravel(order="F")
            B = np.asfortranarray(SB).ravel(order="F")
            got = impl.bf16x3(ta, tb, M, N, K, 1.0, A, SA.shape[0], B, SB.shape[0], 0.0, None, M)
            if not np.array_equal(np.asarray(got, dtype=np.float64), want):
                return False
    return True


def split_closed_form_ok(impl):
    """The split itself, on the table (hi and lo bitwise)."""
    x = np.array([_as_f32(v) for v, _, _ in SPLITS], dtype=np.float32)
    hi, lo = impl.split_bf16(x)
    return (all(F(float(h)) == w for h, (_, w, _) in zip(hi, SPLITS)) and
            all(F(float(l)) == w for l, (_, _, w) in zip(lo, SPLITS)))


# --- scaled FP16: panel exponents ------------------------------------------------

def _panel_case():
    """op(A) 80 x 3 and op(B) 3 x 70 with hand-chosen panel maxima.

    op(A) panels (32 rows): rows 0-15 at most 2^-3 and rows 16-31 holding
    -32 (panel 0: amax 32 = 2^5, and 32 * 2^9 = 2^14, so e = 9); rows 32-63
    zero (e = 0); rows 64-79, the ragged last panel, amax 3 (3 * 2^13 =
    24576 in [2^14, 2^15), so e = 13).  A 16-row grouping would give rows
    0-15 their own exponent 17.
    op(B) panels (32 columns): columns 0-31 amax 1/8 (e = 17), 32-63 amax
    1.5 (e = 14), 64-69 amax 1.75 * 2^-10 (e = 24).
    """
    rng = np.random.default_rng(31)
    opA = np.zeros((80, 3), dtype=np.float32)
    opA[0:16] = rng.uniform(-1, 1, (16, 3)) * 0.125
    opA[3, 1] = -0.125
    opA[16:32] = rng.uniform(-4, 4, (16, 3))
    opA[20, 2] = -32.0
    opA[64:80] = rng.uniform(-2, 2, (16, 3))
    opA[79, 0] = 3.0
    opB = np.zeros((3, 70), dtype=np.float32)
    opB[:, 0:32] = rng.uniform(-0.1, 0.1, (3, 32))
    opB[2, 5] = 0.125
    opB[:, 32:64] = rng.uniform(-1, 1, (3, 32))
    opB[0, 40] = -1.5
    opB[:, 64:70] = rng.uniform(-1, 1, (3, 6)) * 2.0 ** -10
    opB[1, 69] = 1.75 * 2.0 ** -10
    return opA, opB, [9, 0, 13], [17, 14, 24]


def f16_exponents_closed_form_ok(impl):
    opA, opB, eA_want, eB_want = _panel_case()
    M, K = opA.shape
    N = opB.shape[1]
    for ta in "NT":
        for tb in "NT":
            SA = opA.T if ta == "T" else opA
            SB = opB.T if tb == "T" else opB
            ld_a, ld_b = SA.shape[0] + 3, SB.shape[0] + 5
            A = np.full((SA.shape[1], ld_a), np.nan, dtype=np.float32)
            A[:, :SA.shape[0]] = SA.T
            B = np.full((SB.shape[1], ld_b), np.nan, dtype=np.float32)
            B[:, :SB.shape[0]] = SB.T
            eA, eB = impl.f16_exponents(ta, tb, M, N, K, A.ravel(), ld_a, B.ravel(), ld_b)
            if list(np.asarray(eA)) != eA_want or list(np.asarray(eB)) != eB_want:
                return False
    return True


def f16_scaled_subnormal_ok(impl):
    """op(A) 40 x 1: rows 0-15 equal 32, rows 16-39 equal
    a = 2^-25 (1 + 3*2^-10); op(B) = [1, 1] (1 x 2), so op(B)'s exponent is
    14 and fp16(2^14) is exact.

    Rows 16-31 share panel 0 with the 32s, so they are scaled by 2^9:
    a * 2^9 = 2^-16 + 3*2^-26 = 256.75 * 2^-24, below FP16's smallest normal
    2^-14, where the spacing is 2^-24; it rounds to 257 * 2^-24, and the
    unscaled result is 2^-25 + 2^-33.  Rows 32-39 are panel 1 alone,
    amax a, e = 39: a * 2^39 = 2^14 (1 + 3*2^-10) is an FP16 value (spacing
    16 on [2^14, 2^15), and 2^14 * 3*2^-10 = 48), so the result is a.  A
    16-row or 8-row panel, or one exponent for all of op(A), changes one of
    these."""
    a = P ** -25 * (1 + 3 * P ** -10)
    col = [F(32)] * 16 + [P ** -25 + P ** -33] * 16 + [a] * 8
    want = np.array([[float(v), float(v)] for v in col])
    Avals = np.array([32.0] * 16 + [float(a)] * 24, dtype=np.float32)
    assert F(float(Avals[20])) == a
    Bvals = np.ones(2, dtype=np.float32)
    for ta in "NT":
        # op(A) is 40 x 1: stored 40 x 1 (ld 40) for 'N', 1 x 40 (ld 1) for 'T'.
        ld_a = 40 if ta == "N" else 1
        got = impl.f16_scaled(ta, "N", 40, 2, 1, 1.0, Avals, ld_a, Bvals, 1, 0.0, None, 40)
        if not np.array_equal(np.asarray(got, dtype=np.float64), want):
            return False
    return True


def f16_nonfinite_panel_ok(impl):
    """A panel holding Inf or NaN gets exponent 0; its neighbours keep theirs."""
    opA = np.ones((64, 2), dtype=np.float32)
    opA[40, 1] = np.inf
    opB = np.ones((2, 33), dtype=np.float32)
    opB[0, 32] = np.nan
    A = np.asfortranarray(opA).ravel(order="F")
    B = np.asfortranarray(opB).ravel(order="F")
    eA, eB = impl.f16_exponents("N", "N", 64, 33, 2, A, 64, B, 2)
    return list(np.asarray(eA)) == [14, 0] and list(np.asarray(eB)) == [14, 0]


CHECKS = [bf16x3_closed_form_ok, split_closed_form_ok, f16_exponents_closed_form_ok,
          f16_scaled_subnormal_ok, f16_nonfinite_panel_ok]


# --- an independent numpy evaluation, with optional planted mistakes ------------------

def _op(X, ld, trans, rows, cols):
    """op(X) (rows x cols) from a flat column-major buffer."""
    X = np.asarray(X, dtype=np.float32)
    if trans in "Tt":
        return np.array([[X[c + r * ld] for c in range(cols)] for r in range(rows)], np.float32)
    return np.array([[X[r + c * ld] for c in range(cols)] for r in range(rows)], np.float32)


def _stored(X, ld, rows, cols):
    X = np.asarray(X, dtype=np.float32)
    return np.array([[X[r + c * ld] for c in range(cols)] for r in range(rows)], np.float32)


def make_impl(bug=None):
    torch = pytest.importorskip("torch")

    def to_bf16(x):
        x = np.asarray(x, dtype=np.float32)
        if bug == "rz_split":
            return (x.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
        return torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float32).numpy()

    def split_bf16(x):
        x = np.asarray(x, dtype=np.float32)
        hi = to_bf16(x)
        r = (x - hi).astype(np.float32)
        lo = r if bug == "lo_not_rounded" else to_bf16(r)
        return hi, lo

    def bf16x3(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc):
        opA = _op(A, lda, ta, M, K)
        opB = _op(B, ldb, tb, K, N)
        ah, al = split_bf16(opA)
        bh, bl = split_bf16(opB)
        d = lambda x: x.astype(np.float64)
        s = d(ah) @ d(bh) + d(ah) @ d(bl) + d(al) @ d(bh)
        if bug == "keep_lolo":
            s = s + d(al) @ d(bl)
        if bug == "drop_hilo":
            s = s - d(ah) @ d(bl)
        return float(alpha) * s

    panel = 16 if bug == "panel16" else 32

    def expo(amax):
        if not np.isfinite(amax) or amax == 0:
            return 0
        m, p = np.frexp(amax)
        return int((14 if bug == "range_off_by_one" else 15) - p)

    def f16_exponents(ta, tb, M, N, K, A, lda, B, ldb):
        if bug == "stored_orientation":
            SA = _stored(A, lda, *((K, M) if ta in "Tt" else (M, K)))
            SB = _stored(B, ldb, *((N, K) if tb in "Tt" else (K, N)))
            eA = [expo(float(np.max(np.abs(SA[p:p + panel, :])))) for p in range(0, SA.shape[0], panel)]
            eB = [expo(float(np.max(np.abs(SB[:, q:q + panel])))) for q in range(0, SB.shape[1], panel)]
            return np.array(eA), np.array(eB)
        opA = _op(A, lda, ta, M, K).astype(np.float64)
        opB = _op(B, ldb, tb, K, N).astype(np.float64)
        eA = [expo(float(np.max(np.abs(opA[p:p + panel, :])))) for p in range(0, M, panel)]
        eB = [expo(float(np.max(np.abs(opB[:, q:q + panel])))) for q in range(0, N, panel)]
        return np.array(eA), np.array(eB)

    def f16_scaled(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc):
        eA, eB = f16_exponents(ta, tb, M, N, K, A, lda, B, ldb)
        opA = _op(A, lda, ta, M, K)
        opB = _op(B, ldb, tb, K, N)
        rA = np.array([eA[min(i // panel, len(eA) - 1)] for i in range(M)], dtype=np.float64)
        cB = np.array([eB[min(j // panel, len(eB) - 1)] for j in range(N)], dtype=np.float64)
        qA = (opA * np.exp2(rA)[:, None].astype(np.float32)).astype(np.float16).astype(np.float64)
        qB = (opB * np.exp2(cB)[None, :].astype(np.float32)).astype(np.float16).astype(np.float64)
        return float(alpha) * (qA @ qB) * np.exp2(-(rA[:, None] + cB[None, :]))

    return types.SimpleNamespace(split_bf16=split_bf16, bf16x3=bf16x3,
                                 f16_exponents=f16_exponents, f16_scaled=f16_scaled)


BUGS = ["keep_lolo", "rz_split", "drop_hilo", "lo_not_rounded", "panel16",
        "stored_orientation", "range_off_by_one"]


@pytest.mark.parametrize("check", CHECKS, ids=lambda c: c.__name__)
def test_the_oracle_passes(check):
    assert check(oracle)


@pytest.mark.parametrize("check", CHECKS, ids=lambda c: c.__name__)
def test_the_clean_numpy_evaluation_passes(check):
    assert check(make_impl())


@pytest.mark.parametrize("bug", BUGS)
def test_each_planted_mistake_is_caught(bug):
    impl = make_impl(bug)
    failed = [c.__name__ for c in CHECKS if not c(impl)]
    assert failed, "no closed-form pin catches %s" % bug


def test_oracle_panel_width_is_32():
    """The oracle's own panel constant, and the exponent vectors' lengths
    for ragged M and N (ceil(M/32), ceil(N/32))."""
    assert oracle.PANEL == 32
    A = np.ones(65 * 2, dtype=np.float32)
    B = np.ones(2 * 97, dtype=np.float32)
    eA, eB = oracle.f16_exponents("N", "N", 65, 97, 2, A, 65, B, 2)
    assert len(eA) == 3 and len(eB) == 4
