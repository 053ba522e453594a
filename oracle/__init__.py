"""FP64 CPU oracle for C <- alpha*op(A)*op(B) + beta*C (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``, never by the
GPU library.  It shares no code with the GPU path; the only thing both sides
use is the seeded input generator in ``synth``.

Contents
--------
* ``sgemm`` / ``sgemm_entries`` / ``dgemm``: the definition of the Level-3 BLAS
  SGEMM operation (paper, Section 1), the plain three-nested-loop product of
  Section 4 accumulated in FP64 (``oracle.c``).
* ``split_bf16`` and ``bf16x3``: the hi/lo split of an FP32 value into two
  BF16 values and the three-product sum hi*hi + hi*lo + lo*hi, evaluated in
  FP64 (an emulation of the split-precision form; not in the paper).
* ``f16_exponents`` and ``f16_scaled``: power-of-two panel scaling into FP16
  and the scaled product, evaluated in FP64 (not in the paper).
* ``bf16x3_entries`` / ``f16_scaled_entries``: single entries of the two
  forms, for products too large to evaluate whole.
* ``normwise_rel_err`` and ``elementwise_ratio``: error metrics.
* ``dense_grads``: gradients of L = sum((X W) o G) for the dense layer.
* ``mlp_forward`` / ``mlp_loss`` / ``mlp_grads`` / ``mlp_step``: one
  plain-gradient-descent step of a multilayer perceptron, the application the
  paper trains with its SGEMM (Section 4), in FP64 with numpy products.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    """Load liboracle.so, compiling it with gcc first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        i64, f64, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        ch = ctypes.c_char
        L.oracle_sgemm.argtypes = [ch, ch, i64, i64, i64, f64, vp, i64, vp, i64,
                                   f64, vp, i64, vp, i64]
        L.oracle_sgemm_entries.argtypes = [ch, ch, i64, i64, i64, f64, vp, i64, vp,
                                           i64, f64, vp, i64, i64, vp, vp, vp]
        L.oracle_dgemm.argtypes = L.oracle_sgemm.argtypes
        for f in (L.oracle_sgemm, L.oracle_sgemm_entries, L.oracle_dgemm):
            f.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def num_threads():
    """Threads the oracle's parallel loops use."""
    return lib().oracle_num_threads()


def set_num_threads(n):
    """Threads for later oracle calls (results do not depend on it)."""
    lib().oracle_set_num_threads(int(n))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _is_t(t):
    return t in "TtCc"


def _need(buf, dtype, ld, rows, cols, name):
    """Check that a flat column-major buffer covers rows x cols at ld."""
    if buf is None:
        raise ValueError(name + " is None")
    if buf.dtype != dtype or buf.ndim != 1 or not buf.flags.c_contiguous:
        raise ValueError(name + " must be a contiguous 1-D %s array" % dtype)
    if rows > 0 and cols > 0 and buf.size < (cols - 1) * ld + rows:
        raise ValueError(name + " is too small for its shape")


def _check_operands(transA, transB, M, N, K, A, lda, B, ldb, beta, C0, ldc,
                    dtype, use_product):
    if use_product:
        _need(A, dtype, lda, K if _is_t(transA) else M, M if _is_t(transA) else K, "A")
        _need(B, dtype, ldb, N if _is_t(transB) else K, K if _is_t(transB) else N, "B")
    if beta != 0.0:
        _need(C0, dtype, ldc, M, N, "C0")


def sgemm(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc):
    """alpha*op(A)*op(B) + beta*C0 in FP64 from FP32 inputs.

    A, B, C0 are flat float32 arrays in column-major storage with leading
    dimensions lda, ldb, ldc.  Returns an (M, N) float64 array.
    """
    alpha, beta = float(np.float32(alpha)), float(np.float32(beta))
    _check_operands(transA, transB, M, N, K, A, lda, B, ldb, beta, C0, ldc,
                    np.float32, alpha != 0.0 and K > 0)
    out = np.empty((M, N), dtype=np.float64, order="F")
    rc = lib().oracle_sgemm(transA.encode(), transB.encode(), M, N, K, alpha,
                            _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C0), ldc,
                            _ptr(out), max(1, M))
    if rc != 0:
        raise ValueError("oracle_sgemm rejected its arguments (%d)" % rc)
    return out


def sgemm_entries(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc,
                  rows, cols):
    """Only the entries (rows[e], cols[e]) of the FP64 result."""
    alpha, beta = float(np.float32(alpha)), float(np.float32(beta))
    _check_operands(transA, transB, M, N, K, A, lda, B, ldb, beta, C0, ldc,
                    np.float32, alpha != 0.0 and K > 0)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(rows.size, dtype=np.float64)
    rc = lib().oracle_sgemm_entries(transA.encode(), transB.encode(), M, N, K, alpha,
                                    _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C0), ldc,
                                    rows.size, _ptr(rows), _ptr(cols), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_sgemm_entries rejected its arguments (%d)" % rc)
    return out


def dgemm(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc):
    """The same product with FP64 operands (flat float64 arrays)."""
    alpha, beta = float(alpha), float(beta)
    _check_operands(transA, transB, M, N, K, A, lda, B, ldb, beta, C0, ldc,
                    np.float64, alpha != 0.0 and K > 0)
    out = np.empty((M, N), dtype=np.float64, order="F")
    rc = lib().oracle_dgemm(transA.encode(), transB.encode(), M, N, K, alpha,
                            _ptr(A), lda, _ptr(B), ldb, beta, _ptr(C0), ldc,
                            _ptr(out), max(1, M))
    if rc != 0:
        raise ValueError("oracle_dgemm rejected its arguments (%d)" % rc)
    return out


# ---------------------------------------------------------------------------
# Split-precision form: x = hi + lo, both BF16 (round to nearest, ties to even)
# ---------------------------------------------------------------------------

def round_bf16(x):
    """Round FP32 values to the nearest BF16 value, ties to even.

    BF16 keeps the top 16 bits of the FP32 encoding (sign, 8 exponent bits,
    7 fraction bits).  Round-to-nearest-even on the 16 dropped bits: round
    up when they exceed half (0x8000), or equal half and the kept part is
    odd.  Written out on the bit pattern; finite inputs only (an input
    within half a BF16 ulp of FLT_MAX rounds to infinity, as it must).
    """
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    kept = u >> np.uint64(16)
    dropped = u & np.uint64(0xFFFF)
    up = (dropped > 0x8000) | ((dropped == 0x8000) & ((kept & np.uint64(1)) == 1))
    kept = kept + up.astype(np.uint64)
    return (kept << np.uint64(16)).astype(np.uint32).view(np.float32).reshape(np.shape(x))


def split_bf16(x):
    """hi = bf16(x), lo = bf16(x - hi); x - hi is exact in FP32."""
    x = np.asarray(x, dtype=np.float32)
    hi = round_bf16(x)
    lo = round_bf16((x - hi).astype(np.float32))
    return hi, lo


def _split_stored(X):
    """Split a flat stored array (NaN padding stays NaN in hi and lo)."""
    X = np.asarray(X, dtype=np.float32)
    hi, lo = split_bf16(np.where(np.isfinite(X), X, np.float32(0)))
    bad = ~np.isfinite(X)
    hi[bad] = X[bad]
    lo[bad] = X[bad]
    return hi, lo


def bf16x3(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc):
    """alpha*(hiA hiB + hiA loB + loA hiB) + beta*C0, exactly summed in FP64.

    Each term is a product of BF16 values, exact in FP64; the lo*lo term is
    dropped, which is the definition of the three-product split form.
    """
    alpha, beta = float(np.float32(alpha)), float(np.float32(beta))
    Ah, Al = _split_stored(A)
    Bh, Bl = _split_stored(B)
    s = (sgemm(transA, transB, M, N, K, 1.0, Ah, lda, Bh, ldb, 0.0, None, ldc)
         + sgemm(transA, transB, M, N, K, 1.0, Ah, lda, Bl, ldb, 0.0, None, ldc)
         + sgemm(transA, transB, M, N, K, 1.0, Al, lda, Bh, ldb, 0.0, None, ldc))
    out = alpha * s if (alpha != 0.0 and K > 0) else np.zeros((M, N), order="F")
    if beta != 0.0:
        out = out + beta * _logical(C0, ldc, M, N).astype(np.float64)
    return out


def _c0_entries(C0, ldc, rows, cols):
    return np.asarray(C0)[np.asarray(rows, np.int64) + np.asarray(cols, np.int64) * ldc]


def bf16x3_entries(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc, rows, cols):
    """Only the entries (rows[e], cols[e]) of ``bf16x3``, for products too
    large to evaluate whole; the same operations on each entry."""
    alpha, beta = float(np.float32(alpha)), float(np.float32(beta))
    Ah, Al = _split_stored(A)
    Bh, Bl = _split_stored(B)
    e = lambda X, Y: sgemm_entries(transA, transB, M, N, K, 1.0, X, lda, Y, ldb, 0.0, None,
                                   ldc, rows, cols)
    s = e(Ah, Bh) + e(Ah, Bl) + e(Al, Bh)
    out = alpha * s if (alpha != 0.0 and K > 0) else np.zeros(len(rows))
    if beta != 0.0:
        out = out + beta * _c0_entries(C0, ldc, rows, cols).astype(np.float64)
    return out


# ---------------------------------------------------------------------------
# Scaled FP16 form: power-of-two scale per 32-row panel of op(A) and per
# 32-column panel of op(B), taken over the whole K extent
# ---------------------------------------------------------------------------

PANEL = 32


def scale_exponent(amax):
    """The integer e with amax * 2**e in [2**14, 2**15); 0 for amax == 0 or
    a non-finite amax.

    frexp writes amax = f * 2**p with f in [0.5, 1), so amax * 2**(15 - p)
    = f * 2**15 lies in [2**14, 2**15).
    """
    amax = np.asarray(amax, dtype=np.float64)
    _, p = np.frexp(amax)
    e = (15 - p).astype(np.int64)
    ok = np.isfinite(amax) & (amax > 0)
    return np.where(ok, e, 0)


def _logical(X, ld, rows, cols):
    """Stored rows x cols view of a flat column-major buffer as a 2-D array."""
    X = np.asarray(X)
    if rows == 0 or cols == 0:
        return np.zeros((rows, cols), dtype=X.dtype)
    return np.lib.stride_tricks.as_strided(
        X, shape=(rows, cols), strides=(X.itemsize, X.itemsize * ld))


def op_matrix(X, ld, trans, rows, cols):
    """op(X) as a rows x cols float32 array (rows, cols of op(X))."""
    if _is_t(trans):
        return np.array(_logical(X, ld, cols, rows).T, dtype=np.float32)
    return np.array(_logical(X, ld, rows, cols), dtype=np.float32)


def f16_exponents(transA, transB, M, N, K, A, lda, B, ldb):
    """Per-panel exponents: eA[p] for rows 32p..32p+31 of op(A), eB[q] for
    columns 32q..32q+31 of op(B)."""
    opA = op_matrix(A, lda, transA, M, K).astype(np.float64)
    opB = op_matrix(B, ldb, transB, K, N).astype(np.float64)
    eA = np.array([scale_exponent(np.max(np.abs(opA[p:p + PANEL, :]), initial=0.0))
                   for p in range(0, M, PANEL)], dtype=np.int64)
    eB = np.array([scale_exponent(np.max(np.abs(opB[:, q:q + PANEL]), initial=0.0))
                   for q in range(0, N, PANEL)], dtype=np.int64)
    return eA, eB


def _f16_quantised(transA, transB, M, N, K, A, lda, B, ldb):
    """fp16(op(A) 2**eA) and fp16(op(B) 2**eB) as column-major float32
    buffers (leading dimensions M and K), with the per-row exponents of
    op(A) and per-column exponents of op(B).  fp16() rounds to nearest,
    ties to even (numpy's float32 -> float16 conversion)."""
    eA, eB = f16_exponents(transA, transB, M, N, K, A, lda, B, ldb)
    rA = np.repeat(eA, PANEL)[:M]
    cB = np.repeat(eB, PANEL)[:N]
    opA = op_matrix(A, lda, transA, M, K)
    opB = op_matrix(B, ldb, transB, K, N)
    qA = (opA * np.exp2(rA)[:, None].astype(np.float32)).astype(np.float16)
    qB = (opB * np.exp2(cB)[None, :].astype(np.float32)).astype(np.float16)
    qa = np.asfortranarray(qA.astype(np.float32)).ravel(order="F")
    qb = np.asfortranarray(qB.astype(np.float32)).ravel(order="F")
    return qa, qb, rA, cB


def f16_scaled(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc):
    """alpha * 2**-(eA+eB) * fp16(op(A) 2**eA) fp16(op(B) 2**eB) + beta*C0,
    products summed exactly in FP64."""
    alpha, beta = float(np.float32(alpha)), float(np.float32(beta))
    out = np.zeros((M, N), dtype=np.float64, order="F")
    if alpha != 0.0 and K > 0 and M > 0 and N > 0:
        qa, qb, rA, cB = _f16_quantised(transA, transB, M, N, K, A, lda, B, ldb)
        s = sgemm("N", "N", M, N, K, 1.0, qa, max(1, M), qb, max(1, K), 0.0, None, max(1, M))
        out = alpha * s * np.exp2(-(rA[:, None] + cB[None, :]).astype(np.float64))
    if beta != 0.0:
        out = out + beta * _logical(C0, ldc, M, N).astype(np.float64)
    return out


def f16_scaled_entries(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc,
                       rows, cols):
    """Only the entries (rows[e], cols[e]) of ``f16_scaled`` (the exponents
    still come from the whole panels); the same operations on each entry."""
    alpha, beta = float(np.float32(alpha)), float(np.float32(beta))
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    out = np.zeros(rows.size, dtype=np.float64)
    if alpha != 0.0 and K > 0 and M > 0 and N > 0:
        qa, qb, rA, cB = _f16_quantised(transA, transB, M, N, K, A, lda, B, ldb)
        s = sgemm_entries("N", "N", M, N, K, 1.0, qa, max(1, M), qb, max(1, K), 0.0, None,
                          max(1, M), rows, cols)
        out = alpha * s * np.exp2(-(rA[rows] + cB[cols]).astype(np.float64))
    if beta != 0.0:
        out = out + beta * _c0_entries(C0, ldc, rows, cols).astype(np.float64)
    return out


# ---------------------------------------------------------------------------
# Error metrics
# ---------------------------------------------------------------------------

def normwise_rel_err(out, ref):
    """||out - ref||_F / ||ref||_F in FP64 (0 when both are zero)."""
    out = np.asarray(out, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(out - ref)
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return float(num / den)


def abs_product(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc):
    """|alpha| |op(A)| |op(B)| + |beta| |C0|: the scale of the elementwise
    forward-error bound for a matrix product (Higham, Accuracy and Stability
    of Numerical Algorithms, 2nd ed., Section 3.5)."""
    absA = np.abs(np.where(np.isfinite(A), A, 0)).astype(np.float32)
    absB = np.abs(np.where(np.isfinite(B), B, 0)).astype(np.float32)
    return sgemm(transA, transB, M, N, K, abs(float(alpha)), absA, lda, absB, ldb,
                 abs(float(beta)), None if beta == 0 else np.abs(C0).astype(np.float32), ldc)


def elementwise_ratio(out, ref, scale):
    """max_ij |out - ref| / scale (0/0 counts as 0)."""
    d = np.abs(np.asarray(out, dtype=np.float64) - ref)
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(scale > 0, d / scale, np.where(d == 0, 0.0, np.inf))
    return float(np.max(r)) if r.size else 0.0


def gamma(n, u=2.0 ** -24):
    """Higham's gamma_n = n u / (1 - n u)."""
    return n * u / (1.0 - n * u)


# ---------------------------------------------------------------------------
# Dense layer Y = X W, loss L = sum(Y o G): gradients
# ---------------------------------------------------------------------------

def dense_grads(X, W, G):
    """dX = G W^T and dW = X^T G for row-major 2-D float arrays, in FP64.

    X is (B x I), W is (I x O), G is (B x O).  Row-major arrays are handed
    to the column-major oracle as their transposes: a row-major (r x c)
    array is the column-major (c x r) array with leading dimension c.
    """
    X = np.ascontiguousarray(X)
    W = np.ascontiguousarray(W)
    G = np.ascontiguousarray(G)
    nb, ni = X.shape
    no = W.shape[1]
    f = dgemm if X.dtype == np.float64 else sgemm
    xs, ws, gs = X.ravel(), W.ravel(), G.ravel()
    # dX^T (I x B, col-major) = W (I x O) . G^T (O x B): W is col-major (O x I)
    # at ld O, so op = 'T'; G^T is col-major (O x B) at ld O, op = 'N'.
    dXt = f("T", "N", ni, nb, no, 1.0, ws, no, gs, no, 0.0, None, ni)
    # dW^T (O x I) = G^T (O x B) . X (B x I): G^T col-major (O x B) ld O, 'N';
    # X is col-major (I x B) at ld I, its transpose is (B x I): op = 'T'.
    dWt = f("N", "T", no, ni, nb, 1.0, gs, no, xs, ni, 0.0, None, no)
    return np.ascontiguousarray(dXt.T), np.ascontiguousarray(dWt.T)


def dense_loss(X, W, G):
    """L = sum_ij (X W)_ij G_ij in FP64 (FP64 operands)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    nb, ni = X.shape
    no = W.shape[1]
    # Y^T (O x B col-major) = W^T . X^T: W col-major is (O x I) ld O -> 'N';
    # X col-major is (I x B) ld I -> 'N'.
    Yt = dgemm("N", "N", no, nb, ni, 1.0, W.ravel(), no, X.ravel(), ni, 0.0, None, no)
    return float(np.sum(Yt.T * G))


# ---------------------------------------------------------------------------
# Multilayer perceptron (Section 4: a neural network trained with SGEMM as the
# kernel).  The paper names no architecture, loss or update rule; this is the
# reading used here: hidden layers H_l = tanh(H_{l-1} W_l), a linear output
# layer, loss 0.5/B * ||H_L - T||_F^2 over a batch of B rows, and one step of
# plain gradient descent W_l <- W_l - lr dL/dW_l.  Row-major arrays, FP64,
# numpy products; nothing here is blocked or fused.
# ---------------------------------------------------------------------------
def mlp_forward(Ws, X):
    """[H_0 = X, H_1, ..., H_L] in FP64."""
    H = [np.asarray(X, dtype=np.float64)]
    for l, W in enumerate(Ws):
        Z = H[-1] @ np.asarray(W, dtype=np.float64)
        H.append(np.tanh(Z) if l + 1 < len(Ws) else Z)
    return H


def mlp_loss(Ws, X, T):
    """0.5 / B * sum((H_L - T)^2) in FP64."""
    H = mlp_forward(Ws, X)
    E = H[-1] - np.asarray(T, dtype=np.float64)
    return 0.5 * float(np.sum(E * E)) / E.shape[0]


def mlp_grads(Ws, X, T):
    """(loss, [dL/dW_1, ..., dL/dW_L]) by backpropagation in FP64.

    G_L = (H_L - T) / B; dL/dW_l = H_{l-1}^T G_l; and, below the top layer,
    G_{l-1} = (G_l W_l^T) o (1 - H_{l-1}^2), the derivative of tanh.
    """
    H = mlp_forward(Ws, X)
    E = H[-1] - np.asarray(T, dtype=np.float64)
    B = E.shape[0]
    loss = 0.5 * float(np.sum(E * E)) / B
    G = E / B
    dWs = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        dWs[l] = H[l].T @ G
        if l > 0:
            G = (G @ np.asarray(Ws[l], dtype=np.float64).T) * (1.0 - H[l] * H[l])
    return loss, dWs


def mlp_step(Ws, X, T, lr):
    """(loss before the step, [W_l - lr dL/dW_l]) in FP64."""
    loss, dWs = mlp_grads(Ws, X, T)
    return loss, [np.asarray(W, dtype=np.float64) - lr * dW for W, dW in zip(Ws, dWs)]
