"""Cases of tests/golden/integer_cases.json as synth-style dicts (flat
column-major buffers at the stored leading dimensions; padding rows NaN in
A and B and the sentinel in C, as synth lays them out)."""
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "integer_cases.json")


def _buffer(rows_of_cols, ld, pad):
    arr = np.array(rows_of_cols, dtype=np.float32).reshape(len(rows_of_cols), -1)
    rows, cols = arr.shape
    buf = np.full((cols, ld), pad, dtype=np.float32)
    buf[:, :rows] = arr.T
    return buf.reshape(-1)


def golden_cases():
    """(case dict, expected logical C as float64) for each stored case."""
    doc = json.load(open(GOLDEN))
    out = []
    for g in doc["cases"]:
        c = dict(transA=g["transA"], transB=g["transB"], M=g["M"], N=g["N"], K=g["K"],
                 alpha=np.float32(g["alpha"]), beta=np.float32(g["beta"]),
                 A=_buffer(g["A"], g["lda"], np.nan), lda=g["lda"],
                 B=_buffer(g["B"], g["ldb"], np.nan), ldb=g["ldb"],
                 C=_buffer(g["C0"], g["ldc"], synth.C_SENTINEL), ldc=g["ldc"])
        out.append((c, np.array(g["C"], dtype=np.float64)))
    return out
