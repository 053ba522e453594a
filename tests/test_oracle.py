"""Pins for the FP64 oracle: checks against facts that do not come from the
oracle itself (exact rational arithmetic, a library product, closed forms,
invariants).  Each test names the kind of mistake it would catch."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]


def logical(buf, rows, cols, ld):
    """Stored 2-D array from a flat column-major buffer (own code path)."""
    return np.array([[buf[r + c * ld] for c in range(cols)] for r in range(rows)])


def op_rows(buf, trans, rows, cols, ld):
    """op(X) as a Python list of rows, built by an explicit transpose of the
    stored array rather than by index arithmetic."""
    sr, sc = synth.stored_shape(trans, rows, cols)
    S = logical(buf, sr, sc, ld)
    return (S.T if trans in "TtCc" else S).tolist()


# --- brute force with exact rational arithmetic ------------------------------

@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 4), (7, 2, 8), (5, 6, 1), (2, 3, 0)])
def test_brute_force_exact(ta, tb, shape):
    """Catches wrong indices, a transposed operand, a dropped alpha/beta term
    or a wrong sign: the exact value is computed with Fractions."""
    M, N, K = shape
    case = synth.sgemm_case(11 + M * 100 + N * 10 + K, ta, tb, M, N, K,
                            alpha=-1.25, beta=0.75, pad=3)
    got = oracle.sgemm(ta, tb, M, N, K, case["alpha"], case["A"], case["lda"],
                       case["B"], case["ldb"], case["beta"], case["C"], case["ldc"])
    opA = op_rows(case["A"], ta, M, K, case["lda"])
    opB = op_rows(case["B"], tb, K, N, case["ldb"])
    C0 = logical(case["C"], M, N, case["ldc"]).tolist()
    al, be = Fraction(float(case["alpha"])), Fraction(float(case["beta"]))
    for i in range(M):
        for j in range(N):
            s = sum((Fraction(opA[i][k]) * Fraction(opB[k][j]) for k in range(K)), Fraction(0))
            exact = al * s + be * Fraction(C0[i][j])
            mag = abs(float(al)) * sum(abs(opA[i][k] * opB[k][j]) for k in range(K)) \
                + abs(float(be) * C0[i][j])
            assert abs(Fraction(got[i, j]) - exact) <= (K + 2) * 2.0 ** -53 * mag + 1e-300


# --- a library product --------------------------------------------------------

@pytest.mark.parametrize("ta,tb", TRANS)
def test_matches_numpy_float64(ta, tb):
    """A second, independent FP64 product (numpy/BLAS dgemm) on op(A), op(B)
    formed by numpy transposes."""
    M, N, K = 67, 45, 129
    c = synth.sgemm_case(5, ta, tb, M, N, K, alpha=1.5, beta=-0.5)
    got = oracle.sgemm(ta, tb, M, N, K, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                       c["beta"], c["C"], c["ldc"])
    sa = synth.stored_shape(ta, M, K)
    sb = synth.stored_shape(tb, K, N)
    A = c["A"].reshape(sa[1], c["lda"])[:, :sa[0]].T.astype(np.float64)
    B = c["B"].reshape(sb[1], c["ldb"])[:, :sb[0]].T.astype(np.float64)
    C0 = c["C"].reshape(N, c["ldc"])[:, :M].T.astype(np.float64)
    opA = A.T if ta == "T" else A
    opB = B.T if tb == "T" else B
    ref = 1.5 * (opA @ opB) - 0.5 * C0
    assert oracle.normwise_rel_err(got, ref) <= 1e-13


# --- closed forms -------------------------------------------------------------

def test_permutation_gives_permuted_rows_exactly():
    """op(A) = P (a permutation): each output is one exact product, so the
    result is B's rows permuted, bitwise.  Catches a wrong row index."""
    M = K = 9
    N = 5
    rng = np.random.default_rng(3)
    perm = rng.permutation(M)
    P = np.zeros((M, K), dtype=np.float32)
    P[np.arange(M), perm] = 1.0
    A = np.asfortranarray(P).ravel(order="F")
    B = synth.matrix(rng, K, N, K)
    got = oracle.sgemm("N", "N", M, N, K, 1.0, A, M, B, K, 0.0, None, M)
    Bl = B.reshape(N, K).T
    assert np.array_equal(got, Bl[perm, :].astype(np.float64))
    # the same through op(A) = A^T: A stores P^T
    At = np.asfortranarray(P.T).ravel(order="F")
    got_t = oracle.sgemm("T", "N", M, N, K, 1.0, At, K, B, K, 0.0, None, M)
    assert np.array_equal(got_t, got)


def test_k_zero_and_alpha_zero_give_beta_c():
    """K = 0 or alpha = 0: C = beta*C0 exactly and A, B are not read (they
    are NaN here)."""
    M, N = 6, 4
    rng = np.random.default_rng(1)
    C0 = synth.matrix(rng, M, N, M + 2, pad=synth.C_SENTINEL)
    A = np.full(64, np.nan, dtype=np.float32)
    B = np.full(64, np.nan, dtype=np.float32)
    want = (np.float64(-0.5) * C0.reshape(N, M + 2)[:, :M].T.astype(np.float64))
    for K, alpha in ((0, 2.0), (5, 0.0)):
        got = oracle.sgemm("N", "N", M, N, K, alpha, A, M, B, max(1, K), -0.5, C0, M + 2)
        assert np.array_equal(got, want)


def test_beta_zero_does_not_read_c():
    """beta = 0 with NaN in C0: no NaN in the result."""
    c = synth.sgemm_case(2, "N", "N", 8, 8, 8)
    C0 = np.full_like(c["C"], np.nan)
    got = oracle.sgemm("N", "N", 8, 8, 8, 1.0, c["A"], c["lda"], c["B"], c["ldb"], 0.0,
                       C0, c["ldc"])
    assert np.all(np.isfinite(got))


def test_alpha_power_of_two_scales_exactly():
    """alpha = 2**s multiplies the FP64 result by 2**s exactly."""
    c = synth.sgemm_case(4, "T", "N", 17, 13, 33)
    args = ("T", "N", 17, 13, 33)
    one = oracle.sgemm(*args, 1.0, c["A"], c["lda"], c["B"], c["ldb"], 0.0, None, c["ldc"])
    for s in (-3, 5):
        got = oracle.sgemm(*args, 2.0 ** s, c["A"], c["lda"], c["B"], c["ldb"], 0.0, None,
                           c["ldc"])
        assert np.array_equal(got, one * 2.0 ** s)


def test_b_zero_with_beta_one_leaves_c():
    c = synth.sgemm_case(6, "N", "T", 10, 7, 12, beta=1.0)
    Bz = np.zeros_like(c["B"])
    got = oracle.sgemm("N", "T", 10, 7, 12, 3.0, c["A"], c["lda"], Bz, c["ldb"], 1.0,
                       c["C"], c["ldc"])
    assert np.array_equal(got, c["C"].reshape(7, c["ldc"])[:, :10].T.astype(np.float64))


# --- invariants -----------------------------------------------------------------

@pytest.mark.parametrize("ta", ["N", "T"])
def test_row_sum_invariant(ta):
    """B = ones: every column is alpha * the row sums of op(A), compared
    with math.fsum (correctly rounded sum)."""
    M, N, K = 23, 3, 301
    rng = np.random.default_rng(8)
    ra, ca = synth.stored_shape(ta, M, K)
    A = synth.matrix(rng, ra, ca, ra + 5)
    B = np.ones(K * N, dtype=np.float32)
    got = oracle.sgemm(ta, "N", M, N, K, 0.5, A, ra + 5, B, K, 0.0, None, M)
    opA = op_rows(A, ta, M, K, ra + 5)
    for i in range(M):
        want = 0.5 * math.fsum(opA[i])
        tol = K * 2.0 ** -53 * sum(abs(v) for v in opA[i])
        for j in range(N):
            assert abs(got[i, j] - want) <= tol


@pytest.mark.parametrize("ta,tb", TRANS)
def test_integer_inputs_are_exact(ta, tb):
    """Integer entries in [-16, 16]: the result is an exact integer, equal
    to numpy's int64 product."""
    M, N, K = 31, 29, 77
    c = synth.sgemm_case(9, ta, tb, M, N, K, alpha=1.0, beta=1.0, dist="int16",
                         dist_c="int16")
    got = oracle.sgemm(ta, tb, M, N, K, 1.0, c["A"], c["lda"], c["B"], c["ldb"], 1.0,
                       c["C"], c["ldc"])
    A = np.array(op_rows(c["A"], ta, M, K, c["lda"]), dtype=np.int64)
    B = np.array(op_rows(c["B"], tb, K, N, c["ldb"]), dtype=np.int64)
    C0 = logical(c["C"], M, N, c["ldc"]).astype(np.int64)
    assert np.array_equal(got, (A @ B + C0).astype(np.float64))


def test_transpose_consistency():
    """op = T on both sides computes (B A)^T with the same k order as the
    NN product: C_TT(B, A) == C_NN(A, B)^T bitwise."""
    M, N, K = 19, 27, 40
    rng = np.random.default_rng(12)
    A = synth.matrix(rng, M, K, M + 1)
    B = synth.matrix(rng, K, N, K + 2)
    nn = oracle.sgemm("N", "N", M, N, K, 1.0, A, M + 1, B, K + 2, 0.0, None, M)
    tt = oracle.sgemm("T", "T", N, M, K, 1.0, B, K + 2, A, M + 1, 0.0, None, N)
    assert np.array_equal(tt, nn.T)


@pytest.mark.parametrize("ta,tb", TRANS)
def test_padding_is_not_read(ta, tb):
    """NaN padding rows in A and B never reach the result."""
    c = synth.sgemm_case(13, ta, tb, 12, 9, 14, alpha=1.5, beta=-0.5, pad=7)
    got = oracle.sgemm(ta, tb, 12, 9, 14, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                       c["beta"], c["C"], c["ldc"])
    assert np.all(np.isfinite(got))


def test_entries_match_full_result():
    c = synth.sgemm_case(14, "T", "T", 37, 41, 23, alpha=1.5, beta=-0.5)
    full = oracle.sgemm("T", "T", 37, 41, 23, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                        c["beta"], c["C"], c["ldc"])
    r, cc = synth.sample_entries(0, 37, 41, 50)
    part = oracle.sgemm_entries("T", "T", 37, 41, 23, c["alpha"], c["A"], c["lda"], c["B"],
                                c["ldb"], c["beta"], c["C"], c["ldc"], r, cc)
    assert np.array_equal(part, full[r, cc])


@pytest.mark.parametrize("form", ["bf16x3", "f16_scaled"])
def test_form_entries_match_full_result(form):
    """The entry-wise evaluations of the two forms equal the whole-matrix
    ones bitwise, sampled corners and ragged panels included."""
    full_fn = getattr(oracle, form)
    part_fn = getattr(oracle, form + "_entries")
    for ta, tb in TRANS:
        c = synth.sgemm_case(16, ta, tb, 70, 41, 23, alpha=1.5, beta=-0.5, dist="loguni")
        a = (ta, tb, 70, 41, 23, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"], c["beta"],
             c["C"], c["ldc"])
        full = full_fn(*a)
        r, cc = synth.sample_entries(1, 70, 41, 60)
        assert np.array_equal(part_fn(*a, r, cc), full[r, cc])


def test_dgemm_equals_sgemm_on_float32_values():
    c = synth.sgemm_case(15, "N", "T", 16, 18, 20, alpha=1.5, beta=-0.5)
    s = oracle.sgemm("N", "T", 16, 18, 20, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"],
                     c["beta"], c["C"], c["ldc"])
    d = oracle.dgemm("N", "T", 16, 18, 20, 1.5, c["A"].astype(np.float64), c["lda"],
                     c["B"].astype(np.float64), c["ldb"], -0.5,
                     c["C"].astype(np.float64), c["ldc"])
    assert np.array_equal(s, d)


def test_rejects_bad_arguments():
    A = np.zeros(16, dtype=np.float32)
    with pytest.raises(ValueError):
        oracle.sgemm("X", "N", 2, 2, 2, 1.0, A, 2, A, 2, 0.0, None, 2)
    with pytest.raises(ValueError):
        oracle.sgemm("N", "N", 4, 2, 2, 1.0, A, 2, A, 2, 0.0, None, 4)  # lda < M


# --- the BF16 hi/lo split -----------------------------------------------------------

def test_round_bf16_matches_torch():
    """Round-to-nearest-even into BF16 agrees with torch's conversion, on
    random values and on constructed ties."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.uniform(-4, 4, 20000).astype(np.float32),
        np.exp2(rng.uniform(-100, 100, 5000)).astype(np.float32),
        # ties: kept part even (stays) and odd (rounds up)
        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 2 ** -120 * (1 + 2 ** -8)],
                 dtype=np.float32),
    ])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(oracle.round_bf16(x), want)
    assert oracle.round_bf16(np.float32(1 + 2 ** -8)) == np.float32(1.0)
    assert oracle.round_bf16(np.float32(1 + 3 * 2 ** -8)) == np.float32(1 + 2 ** -6)


def test_split_reconstructs_to_2_pow_minus_16():
    rng = np.random.default_rng(1)
    x = (rng.uniform(-1, 1, 100000) * np.exp2(rng.uniform(-20, 20, 100000))).astype(np.float32)
    hi, lo = oracle.split_bf16(x)
    for v in (hi, lo):  # both halves are BF16 values: low 16 bits zero
        assert np.all((v.view(np.uint32) & 0xFFFF) == 0)
    err = np.abs(x.astype(np.float64) - hi - lo)
    assert np.all(err <= 2.0 ** -16 * np.abs(x))
    # hi alone is much worse: the lo part is doing real work
    assert np.max(np.abs(x - hi) / np.abs(x)) > 2.0 ** -10


def test_bf16x3_is_exact_on_small_integers():
    """|v| <= 16 is a BF16 value, so lo = 0 and the form equals the oracle."""
    c = synth.sgemm_case(21, "T", "N", 33, 35, 70, alpha=1.0, beta=1.0, dist="int16",
                         dist_c="int16")
    a = (c["transA"], c["transB"], 33, 35, 70, 1.0, c["A"], c["lda"], c["B"], c["ldb"], 1.0,
         c["C"], c["ldc"])
    assert np.array_equal(oracle.bf16x3(*a), oracle.sgemm(*a))


def test_bf16x3_error_is_split_sized():
    """Dropping the hi*lo or lo*hi term would leave a ~1e-3 error; dropping
    nothing leaves the lo*lo term and the split residue, ~1e-5 or less."""
    M = N = K = 96
    c = synth.sgemm_case(22, "N", "N", M, N, K)
    a = ("N", "N", M, N, K, 1.0, c["A"], c["lda"], c["B"], c["ldb"], 0.0, None, c["ldc"])
    err = oracle.normwise_rel_err(oracle.bf16x3(*a), oracle.sgemm(*a))
    assert 1e-8 < err < 1e-5


# --- FP16 power-of-two panel scaling ----------------------------------------------

def test_scale_exponent_closed_forms():
    assert oracle.scale_exponent(1.0) == 14
    assert oracle.scale_exponent(1.5) == 14
    assert oracle.scale_exponent(2.0) == 13
    assert oracle.scale_exponent(2.0 ** -8) == 22
    assert oracle.scale_exponent(2.0 ** 8 * 1.999) == 6
    assert oracle.scale_exponent(0.0) == 0
    assert oracle.scale_exponent(np.inf) == 0
    assert oracle.scale_exponent(np.nan) == 0
    rng = np.random.default_rng(2)
    amax = np.exp2(rng.uniform(-30, 30, 1000))
    e = oracle.scale_exponent(amax)
    scaled = amax * np.exp2(e.astype(np.float64))
    assert np.all((scaled >= 2.0 ** 14) & (scaled < 2.0 ** 15))


def test_f16_scaled_is_exact_on_small_integers():
    """Integers scaled by a power of two stay exact in FP16, so the unscaled
    result equals the oracle exactly (a wrong unscale exponent fails)."""
    c = synth.sgemm_case(23, "N", "T", 70, 45, 66, alpha=2.0, beta=-1.0, dist="int16",
                         dist_c="int16")
    a = ("N", "T", 70, 45, 66, 2.0, c["A"], c["lda"], c["B"], c["ldb"], -1.0, c["C"], c["ldc"])
    assert np.array_equal(oracle.f16_scaled(*a), oracle.sgemm(*a))


def test_f16_scaled_identity_quantises_b_only():
    """op(A) = I: the result is B rounded to FP16 after scaling, so every
    element is within 2**-11 relative of B."""
    K = M = 64
    N = 40
    rng = np.random.default_rng(5)
    A = np.eye(M, dtype=np.float32).ravel(order="F")
    B = synth.matrix(rng, K, N, K, dist="loguni")
    got = oracle.f16_scaled("N", "N", M, N, K, 1.0, A, M, B, K, 0.0, None, M)
    Bl = B.reshape(N, K).T.astype(np.float64)
    assert np.all(np.abs(got - Bl) <= 2.0 ** -11 * np.abs(Bl))
    assert np.any(got != Bl)


def test_f16_scaled_error_on_wide_range_inputs():
    """Sign-random magnitudes 2**U[-8, 8]: the scaled FP16 form stays within
    1e-3 normwise of the FP64 product (an unscaled FP16 cast would not
    overflow here, but a missing unscale would be off by 2**28)."""
    M = N = K = 128
    c = synth.sgemm_case(24, "N", "N", M, N, K, dist="loguni")
    a = ("N", "N", M, N, K, 1.0, c["A"], c["lda"], c["B"], c["ldb"], 0.0, None, c["ldc"])
    err = oracle.normwise_rel_err(oracle.f16_scaled(*a), oracle.sgemm(*a))
    assert 1e-6 < err < 1e-3


# --- dense layer gradients ------------------------------------------------------------

def test_dense_grads_match_finite_differences():
    """L = sum((X W) o G) is linear in each of X and W, so a central
    difference equals the derivative up to FP64 rounding."""
    X, W, G = synth.dense_layer(0, 64, 48, 32)
    X, W, G = (v.astype(np.float64) for v in (X, W, G))
    dX, dW = oracle.dense_grads(X, W, G)
    rng = np.random.default_rng(7)
    h = 1e-3
    for _ in range(24):
        i, k = rng.integers(0, 64), rng.integers(0, 48)
        Xp, Xm = X.copy(), X.copy()
        Xp[i, k] += h
        Xm[i, k] -= h
        fd = (oracle.dense_loss(Xp, W, G) - oracle.dense_loss(Xm, W, G)) / (2 * h)
        assert abs(fd - dX[i, k]) <= 1e-9 * max(1.0, abs(dX[i, k]))
        k2, j = rng.integers(0, 48), rng.integers(0, 32)
        Wp, Wm = W.copy(), W.copy()
        Wp[k2, j] += h
        Wm[k2, j] -= h
        fd = (oracle.dense_loss(X, Wp, G) - oracle.dense_loss(X, Wm, G)) / (2 * h)
        assert abs(fd - dW[k2, j]) <= 1e-9 * max(1.0, abs(dW[k2, j]))


def test_dense_grads_match_numpy():
    X, W, G = synth.dense_layer(1, 40, 24, 36)
    dX, dW = oracle.dense_grads(X, W, G)
    X64, W64, G64 = (v.astype(np.float64) for v in (X, W, G))
    assert oracle.normwise_rel_err(dX, G64 @ W64.T) <= 1e-13
    assert oracle.normwise_rel_err(dW, X64.T @ G64) <= 1e-13


def test_dense_loss_matches_numpy():
    X, W, G = (v.astype(np.float64) for v in synth.dense_layer(4, 20, 12, 16))
    want = float(np.sum((X @ W) * G))
    assert abs(oracle.dense_loss(X, W, G) - want) <= 1e-12 * max(1.0, abs(want))


def test_results_do_not_depend_on_thread_count():
    """Every output is one sequential dot product, so the thread count can
    only change who computes it: bitwise equal at 1 thread and at the
    default count."""
    c = synth.sgemm_case(77, "T", "N", 70, 130, 90, alpha=1.5, beta=-0.5, pad=3)
    args = (c["transA"], c["transB"], c["M"], c["N"], c["K"], c["alpha"], c["A"], c["lda"],
            c["B"], c["ldb"], c["beta"], c["C"], c["ldc"])
    default = oracle.num_threads()
    many = oracle.sgemm(*args)
    try:
        oracle.set_num_threads(1)
        assert oracle.num_threads() == 1
        one = oracle.sgemm(*args)
    finally:
        oracle.set_num_threads(default)
    assert np.array_equal(one, many)


def test_golden_integer_cases():
    """The stored exact results (tests/golden, checked against Fractions
    when they were written) are reproduced bitwise."""
    from golden_util import golden_cases
    cases = golden_cases()
    assert len(cases) == 6
    for c, want in cases:
        got = oracle.sgemm(c["transA"], c["transB"], c["M"], c["N"], c["K"], c["alpha"], c["A"],
                           c["lda"], c["B"], c["ldb"], c["beta"], c["C"], c["ldc"])
        assert np.array_equal(got, want)
