"""Hardware numerics the tolerances rest on, probed through the public API.

* MFMA FP32 accumulation rounding: the elementwise bound used everywhere
  (gamma with u = 2**-23) covers any rounding mode; these cases pin the mode
  actually observed -- round to nearest, ties to even -- so a change (a
  different instruction, a truncating accumulate) is noticed.
* Denormals: FP32 denormal inputs and denormal results pass through every
  form unchanged (no flush to zero).
"""
import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu

U = 2.0 ** -23


def dot(a, b, prec="fp32"):
    """C(1x1) = a . b through sgemm NN with M = N = 1, K = len(a)."""
    import torch
    import paper_1912_04379_amd as mg
    K = len(a)
    A = torch.tensor(np.array(a, np.float32), device="cuda")
    B = torch.tensor(np.array(b, np.float32), device="cuda")
    C = torch.zeros(1, device="cuda")
    mg.sgemm("N", "N", 1, 1, K, 1.0, A, 1, B, K, 0.0, C, 1, precision=prec)
    torch.cuda.synchronize()
    return float(C.cpu()[0])


# (a, b, round-to-nearest-even result); round toward zero differs in each
# case except the ties, which separate ties-to-even from ties-away.
ROUNDING = {
    "1 + 3/4 ulp": ([1.0, 3 * 2.0 ** -25], [1.0, 1.0], 1 + U),
    "1 + 1/4 ulp": ([1.0, 2.0 ** -25], [1.0, 1.0], 1.0),
    "1 + 1/2 ulp, tie to even (down)": ([1.0, 2.0 ** -24], [1.0, 1.0], 1.0),
    "1 + ulp + 1/2 ulp, tie to even (up)": ([1.0 + U, 2.0 ** -24], [1.0, 1.0], 1 + 2 * U),
    "-(1 + 3/4 ulp)": ([-1.0, -3 * 2.0 ** -25], [1.0, 1.0], -(1 + U)),
    # k = 0 and k = 8 of a 16-deep slab meet inside one MFMA instruction
    "one instruction, 1 + 3/4 ulp": ([1.0] + [0.0] * 7 + [3 * 2.0 ** -25] + [0.0] * 7,
                                     [1.0] * 16, 1 + U),
}


@pytest.mark.parametrize("name", list(ROUNDING))
def test_fp32_mfma_accumulation_rounds_to_nearest_even(name):
    a, b, want = ROUNDING[name]
    got = dot(a, b)
    log("rounding %s: %r" % (name, got))
    assert got == want


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16s"])
@pytest.mark.parametrize("a,b", [(2.0 ** -130, 2.0 ** 10),    # denormal input
                                 (2.0 ** -100, 2.0 ** -30),   # denormal result
                                 (2.0 ** -126, 0.5)])          # min normal / 2
def test_denormals_are_kept(prec, a, b):
    want = float(np.float32(a) * np.float32(b))
    got = dot([a], [b], prec)
    log("%s %r * %r = %r" % (prec, a, b, got))
    assert got == want and got != 0.0
