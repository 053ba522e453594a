"""Write tests/golden/integer_cases.json: small SGEMM problems with integer
inputs and their results (C <- alpha op(A) op(B) + beta C, Section 1).

The paper prints no worked example, so the stored results come from the
oracle (`oracle.sgemm`), and this script first checks each one against the
exact rational value of the definition (Python Fractions).  With integer
entries in [-16, 16], integer alpha and beta, and K <= 16, every partial sum
is an integer far below 2**24: exact in FP32, in the BF16 split (hi = x,
lo = 0) and in scaled FP16, so every form of the library must reproduce
these results bitwise.

    python tests/golden/make_golden.py
"""
import json
import os
import sys
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

# (transA, transB, M, N, K, alpha, beta, pad); seeds are the case numbers
CASES = [("N", "N", 3, 4, 5, 1, 0, 0), ("N", "T", 5, 3, 7, 2, -1, 2), ("T", "N", 4, 6, 3, -1, 3, 1),
         ("T", "T", 7, 5, 16, 3, 1, 4), ("N", "N", 33, 1, 9, 1, -2, 3), ("T", "N", 1, 40, 11, -2, 0, 0)]


def stored(buf, rows, cols, ld):
    return [[float(buf[r + c * ld]) for c in range(cols)] for r in range(rows)]


def exact(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc):
    opA = (lambda i, k: A[k + i * lda]) if ta == "T" else (lambda i, k: A[i + k * lda])
    opB = (lambda k, j: B[j + k * ldb]) if tb == "T" else (lambda k, j: B[k + j * ldb])
    out = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            s = sum((Fraction(float(opA(i, k))) * Fraction(float(opB(k, j))) for k in range(K)),
                    Fraction(0))
            v = Fraction(alpha) * s + Fraction(beta) * Fraction(float(C[i + j * ldc]))
            out[i, j] = float(v)
            assert Fraction(out[i, j]) == v          # representable exactly
    return out


def main():
    cases = []
    for n, (ta, tb, M, N, K, alpha, beta, pad) in enumerate(CASES):
        c = synth.sgemm_case(100 + n, ta, tb, M, N, K, alpha=alpha, beta=beta, pad=pad,
                             dist="int16", dist_c="int16")
        args = (ta, tb, M, N, K, c["alpha"], c["A"], c["lda"], c["B"], c["ldb"], c["beta"],
                c["C"], c["ldc"])
        got = oracle.sgemm(*args)
        want = exact(ta, tb, M, N, K, alpha, c["A"], c["lda"], c["B"], c["ldb"], beta, c["C"],
                     c["ldc"])
        assert np.array_equal(got, want), "oracle differs from the exact value"
        ra, ca = synth.stored_shape(ta, M, K)
        rb, cb = synth.stored_shape(tb, K, N)
        cases.append(dict(transA=ta, transB=tb, M=M, N=N, K=K, alpha=alpha, beta=beta,
                          lda=c["lda"], ldb=c["ldb"], ldc=c["ldc"],
                          A=stored(c["A"], ra, ca, c["lda"]), B=stored(c["B"], rb, cb, c["ldb"]),
                          C0=stored(c["C"], M, N, c["ldc"]), C=got.tolist()))
    doc = {"what": "C <- alpha op(A) op(B) + beta C (Section 1) on integer inputs; arrays are the "
                   "referenced stored rows x columns (column index second); C is the logical M x N "
                   "result", "cases": cases}
    with open(os.path.join(HERE, "integer_cases.json"), "w") as f:
        json.dump(doc, f, indent=None, separators=(",", ":"))
        f.write("\n")
    print("wrote %d cases" % len(cases))


if __name__ == "__main__":
    main()
