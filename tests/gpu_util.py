"""Helpers for GPU parity tests: upload a seeded case, run the library on
it, and compare with the FP64 oracle."""
import sys

import numpy as np

import oracle
import paper_1912_04379_amd as mg
import synth

U = 2.0 ** -24


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(buf):
    import torch
    if buf is None or buf.size == 0:
        return torch.empty(1, dtype=torch.float32, device="cuda")
    return torch.from_numpy(np.ascontiguousarray(buf)).to("cuda")


def run(case, precision="fp32", config=-1, stream=None):
    """Run the library on a synth case; returns the whole C buffer (numpy),
    padding included."""
    import torch
    A, B, C = to_dev(case["A"]), to_dev(case["B"]), to_dev(case["C"])
    mg.sgemm(case["transA"], case["transB"], case["M"], case["N"], case["K"],
             float(case["alpha"]), A, case["lda"], B, case["ldb"], float(case["beta"]), C,
             case["ldc"], precision=precision, config=config, stream=stream)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:case["C"].size]


# Leading dimension (floats) beyond which byte offsets inside one column
# block no longer fit the 32-bit buffer addressing: the library switches to
# 64-bit addresses there.
WIDE_LD = 2 ** 21 + 3


def wide_ldc_case(seed, ta, tb, M, N, K, **kw):
    """A synth case whose C has leading dimension WIDE_LD (keep N small:
    the C buffer holds N * WIDE_LD floats)."""
    c = synth.sgemm_case(seed, ta, tb, M, N, K, pad=3, **kw)
    rng = np.random.default_rng(seed + 1)
    c["C"] = synth.matrix(rng, M, N, WIDE_LD, pad=synth.C_SENTINEL)
    c["ldc"] = WIDE_LD
    return c


def logical_c(cbuf, case):
    M, N, ldc = case["M"], case["N"], case["ldc"]
    return cbuf.reshape(N, ldc)[:, :M].T.astype(np.float64)


def padding_untouched(cbuf, case):
    M, N, ldc = case["M"], case["N"], case["ldc"]
    if ldc == M or N == 0:
        return True
    pad = cbuf.reshape(N, ldc)[:, M:]
    return bool(np.all(pad == synth.C_SENTINEL))


def oracle_args(case):
    return (case["transA"], case["transB"], case["M"], case["N"], case["K"], case["alpha"],
            case["A"], case["lda"], case["B"], case["ldb"], case["beta"], case["C"],
            case["ldc"])


def fp32_bound(case):
    """Elementwise bound for any correctly rounded FP32 evaluation order:
    gamma_{K+2} |alpha| |op(A)||op(B)| + 2u |beta C0| (Higham, Section 3.5),
    with u = 2**-23 so that directed rounding inside the MFMA is covered."""
    scale = oracle.abs_product(*oracle_args(case))
    return oracle.gamma(case["K"] + 2, 2.0 ** -23) * scale


def full_check(case, got_buf, bound_fn=fp32_bound, normwise=1e-5):
    ref = oracle.sgemm(*oracle_args(case))
    got = logical_c(got_buf, case)
    assert padding_untouched(got_buf, case), "C padding was written"
    assert np.all(np.isfinite(got)), "non-finite output"
    err = oracle.normwise_rel_err(got, ref)
    assert err <= normwise, "normwise error %.3e > %.1e" % (err, normwise)
    if bound_fn is not None:
        bound = bound_fn(case)
        viol = np.abs(got - ref) > bound
        assert not viol.any(), "elementwise bound violated at %s" % (np.argwhere(viol)[:5],)
    return err


def sampled_check(case, got_buf, count=3000, seed=0, bound_fn=fp32_bound, normwise=1e-5):
    """Check sampled entries (oracle one by one) at sizes too big for the
    full oracle; padding and finiteness are checked everywhere."""
    M, N = case["M"], case["N"]
    rows, cols = synth.sample_entries(seed, M, N, count)
    ref = oracle.sgemm_entries(*oracle_args(case), rows, cols)
    C = got_buf.reshape(N, case["ldc"])
    got = C[cols, rows].astype(np.float64)
    assert padding_untouched(got_buf, case), "C padding was written"
    assert np.all(np.isfinite(C[:, :M])), "non-finite output"
    err = oracle.normwise_rel_err(got, ref)
    assert err <= normwise, "sampled normwise error %.3e" % err
    if bound_fn is not None:
        # bound on the sampled entries only
        absA = np.abs(np.where(np.isfinite(case["A"]), case["A"], 0)).astype(np.float32)
        absB = np.abs(np.where(np.isfinite(case["B"]), case["B"], 0)).astype(np.float32)
        absC = np.abs(case["C"]).astype(np.float32)
        scale = oracle.sgemm_entries(case["transA"], case["transB"], M, N, case["K"],
                                     abs(float(case["alpha"])), absA, case["lda"], absB,
                                     case["ldb"], abs(float(case["beta"])), absC, case["ldc"],
                                     rows, cols)
        bound = bound_fn.sampled(case, scale) if hasattr(bound_fn, "sampled") else \
            oracle.gamma(case["K"] + 2, 2.0 ** -23) * scale
        assert np.all(np.abs(got - ref) <= bound), "elementwise bound violated"
    return err
