"""Seeded synthetic inputs for the SGEMM library and its oracle.

This module is shared by the GPU tests, the benchmark and the oracle-side
tests.  It only draws random numbers and lays them out in memory; it holds
none of the product's arithmetic.

Storage is column-major: a stored array of ``rows`` x ``cols`` with leading
dimension ``ld`` is a flat float32 buffer of ``ld * cols`` values, element
(r, c) at ``r + c*ld``.  Rows ``rows .. ld-1`` of every column are padding:
NaN in A and B (a kernel that reads them poisons its result) and the
sentinel ``C_SENTINEL`` in C (a kernel that writes them is caught).

Random streams: ``numpy.random.default_rng(seed)`` (PCG64).  For one GEMM
the draws are made in the order A, B, C, each over its stored array in
column-major order, as float64 values cast to float32 (round to nearest).
"""
import numpy as np

C_SENTINEL = np.float32(7.0e30)


def is_trans(t):
    if t not in "NnTtCc" or len(t) != 1:
        raise ValueError("trans flag must be one of N, T, C")
    return t in "TtCc"


def stored_shape(trans, rows, cols):
    """Stored (rows, cols) of an operand whose op() is rows x cols."""
    return (cols, rows) if is_trans(trans) else (rows, cols)


def draw(rng, n, dist):
    """n values from one of the input distributions.

    uniform:  i.i.d. uniform on [-1, 1).
    loguni:   sign-random magnitude 2**U[-8, 8]: all n signs are drawn
              first, then all n exponents.
    int16:    integers uniform on [-16, 16] (exact in FP32, BF16 and FP16,
              and every partial sum below 2**24 stays exact in FP32).
    ones:     all ones (no draw).
    """
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=n)
    if dist == "loguni":
        sign = np.where(rng.integers(0, 2, size=n) == 0, -1.0, 1.0)
        expo = rng.uniform(-8.0, 8.0, size=n)
        return sign * np.exp2(expo)
    if dist == "int16":
        return rng.integers(-16, 17, size=n).astype(np.float64)
    if dist == "ones":
        return np.ones(n)
    raise ValueError("unknown distribution " + repr(dist))


def matrix(rng, rows, cols, ld, dist="uniform", pad=np.nan):
    """Flat float32 column-major stored array with padding rows."""
    if ld < max(1, rows):
        raise ValueError("ld must be >= max(1, rows)")
    buf = np.full((max(cols, 0), ld), pad, dtype=np.float32)
    vals = draw(rng, rows * cols, dist).astype(np.float32)
    buf[:, :rows] = vals.reshape(cols, rows)
    return buf.reshape(-1)


def sgemm_case(seed, transA, transB, M, N, K, *, alpha=1.0, beta=0.0,
               pad=16, dist="uniform", dist_c="uniform"):
    """One SGEMM problem: dict with A, lda, B, ldb, C, ldc and the scalars.

    Leading dimensions are the stored rows plus ``pad`` (the paper times
    with a fixed stride larger than the row length, Section 4).  C holds
    the initial C0.
    """
    rng = np.random.default_rng(seed)
    ra, ca = stored_shape(transA, M, K)
    rb, cb = stored_shape(transB, K, N)
    lda, ldb, ldc = max(1, ra + pad), max(1, rb + pad), max(1, M + pad)
    A = matrix(rng, ra, ca, lda, dist)
    B = matrix(rng, rb, cb, ldb, dist)
    C = matrix(rng, M, N, ldc, dist_c, pad=C_SENTINEL)
    return dict(transA=transA, transB=transB, M=M, N=N, K=K,
                alpha=np.float32(alpha), beta=np.float32(beta),
                A=A, lda=lda, B=B, ldb=ldb, C=C, ldc=ldc)


def grouped_problems(seed=0, count=512, lo=16, hi=512):
    """Shapes for a batch of independent GEMMs.

    For each problem, in order: M, N, K uniform on {lo..hi} (inclusive),
    then transA 'N' or 'T' with probability 1/2; transB is 'N'.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        M, N, K = (int(v) for v in rng.integers(lo, hi + 1, size=3))
        ta = "T" if rng.integers(0, 2) == 1 else "N"
        out.append(dict(transA=ta, transB="N", M=M, N=N, K=K))
    return out


def grouped_data(problems, seed=1, dist="uniform"):
    """Operands for ``grouped_problems``: tight leading dimensions (stored
    rows), drawn per problem in the order A, B, C from one stream."""
    rng = np.random.default_rng(seed)
    data = []
    for p in problems:
        ra, ca = stored_shape(p["transA"], p["M"], p["K"])
        rb, cb = stored_shape(p["transB"], p["K"], p["N"])
        A = matrix(rng, ra, ca, max(1, ra), dist)
        B = matrix(rng, rb, cb, max(1, rb), dist)
        C = matrix(rng, p["M"], p["N"], max(1, p["M"]), dist)
        data.append(dict(A=A, lda=max(1, ra), B=B, ldb=max(1, rb), C=C, ldc=max(1, p["M"])))
    return data


def dense_layer(seed, batch, n_in, n_out):
    """X (batch x n_in), W (n_in x n_out), G (batch x n_out), row-major
    float32, uniform on [-1, 1), drawn in the order X, W, G."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(batch, n_in)).astype(np.float32)
    W = rng.uniform(-1.0, 1.0, size=(n_in, n_out)).astype(np.float32)
    G = rng.uniform(-1.0, 1.0, size=(batch, n_out)).astype(np.float32)
    return X, W, G


def mlp_case(seed, batch, widths):
    """Inputs of a multilayer-perceptron training step, row-major float32,
    drawn in the order X, T, W_1 .. W_L.

    X (batch x widths[0]) and the targets T (batch x widths[-1]) are
    uniform on [-1, 1); W_l (widths[l-1] x widths[l]) is uniform on
    [-1, 1) times sqrt(3 / widths[l-1]), so each unit's input has about the
    variance of one input value and tanh is not saturated.
    """
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, size=(batch, widths[0])).astype(np.float32)
    T = rng.uniform(-1.0, 1.0, size=(batch, widths[-1])).astype(np.float32)
    Ws = [(rng.uniform(-1.0, 1.0, size=(a, b)) * np.sqrt(3.0 / a)).astype(np.float32)
          for a, b in zip(widths[:-1], widths[1:])]
    return X, T, Ws


def sample_entries(seed, M, N, count):
    """Seeded (row, col) positions for checking single outputs of a large
    product: the four corners and the last row/column are always included
    (ragged tiles sit there), the rest uniform."""
    rng = np.random.default_rng(seed)
    r = list(rng.integers(0, M, size=count))
    c = list(rng.integers(0, N, size=count))
    fixed = [(0, 0), (M - 1, 0), (0, N - 1), (M - 1, N - 1)]
    fixed += [(M - 1, int(j)) for j in rng.integers(0, N, size=8)]
    fixed += [(int(i), N - 1) for i in rng.integers(0, M, size=8)]
    for i, j in fixed:
        r.append(i)
        c.append(j)
    return np.array(r, dtype=np.int64), np.array(c, dtype=np.int64)
