"""Error bars for the two 16-bit forms against the oracle's FP64 emulation
of the same form (same splits and scalings, exact sums).

The GPU result differs from that emulation only by FP32 rounding: one
rounding of the accumulator per MFMA block of products, and the
alpha/beta epilogue.  Two bars:

* elementwise, valid for any order and for directed rounding inside the
  MFMA: gamma_n(2**-23) times the sum of the magnitudes of the terms
  (Higham, Accuracy and Stability of Numerical Algorithms, 2nd ed.,
  Section 3.5), n = 3K + 2 (three products per k) or K + 2;
* normwise and statistical, for round-to-nearest accumulation with errors
  of random sign: ||got - emu||_F / ||emu||_F <= 2**-24 (STAT_C sqrt(K) + 2).
  The sqrt(K) term is the random walk of the accumulator roundings, the 2
  the epilogue's two roundings.  A numpy model of the kernels'
  accumulation (16 products per rounding) measures 0.08 to 0.14 sqrt(K)
  u on uniform and wide-range inputs; a truncating split, a dropped
  correction term, a kept lo*lo (at K <= 2048) or a truncating FP16
  conversion each exceed the bar (tests/test_form_bar.py shows it).
"""
import math

STAT_C = 0.5
U = 2.0 ** -24


def stat_bar(K):
    """Normwise bar of the GPU result against the form's FP64 emulation."""
    return U * (STAT_C * math.sqrt(max(int(K), 1)) + 2.0)
