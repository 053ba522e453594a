"""Pre-packed op(B) (BF16x3 and scaled FP16): products with a packed B
equal the ordinary call of the same form on the same packed configuration
bitwise (the same packed values and exponents reach the same kernel), and
the FP64 oracle within the form's bar (1e-5 BF16x3, 1e-3 FP16); one handle
serves several products.  FP32: op(B) transposed once into a k-contiguous
K x N array; products equal the ordinary call with op(B) given as a stored
K x N 'N' operand bitwise, and the oracle within the FP32 elementwise
bound."""
import numpy as np
import pytest

import oracle
import synth
import paper_1912_04379_amd as mg
from gpu_util import full_check, log, logical_c, oracle_args, to_dev, wide_ldc_case

pytestmark = pytest.mark.gpu

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]
PRECS = ["bf16x3", "fp16s"]
BAR = {"bf16x3": 1e-5, "fp16s": 1e-3}


def packed_config(M, N):
    """16-bit configuration the packed-B call runs: pipelined 256 x 256 from
    144 such tiles, else pipelined 128 x 128."""
    return 10 if ((M + 255) // 256) * ((N + 255) // 256) >= 144 else 11


def both(c, prec):
    """(result of the ordinary call, result with a packed B), whole C
    buffers."""
    import torch
    A, B = to_dev(c["A"]), to_dev(c["B"])
    C1, C2 = to_dev(c["C"]), to_dev(c["C"])
    M, N, K = c["M"], c["N"], c["K"]
    mg.sgemm(c["transA"], c["transB"], M, N, K, float(c["alpha"]), A, c["lda"], B, c["ldb"],
             float(c["beta"]), C1, c["ldc"], precision=prec, config=packed_config(M, N))
    with mg.PackedB(c["transB"], K, N, B, c["ldb"], precision=prec) as pb:
        pb.sgemm(c["transA"], M, float(c["alpha"]), A, c["lda"], float(c["beta"]), C2, c["ldc"])
    torch.cuda.synchronize()
    return C1.cpu().numpy(), C2.cpu().numpy()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", [(300, 270, 77), (513, 257, 1000), (33, 65, 7), (1, 1, 1)])
def test_equals_ordinary_call_and_oracle(prec, ta, tb, shape):
    M, N, K = shape
    c = synth.sgemm_case(51, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3)
    log("packed B %s %s %s%s" % (prec, shape, ta, tb))
    ref_buf, got_buf = both(c, prec)
    assert np.array_equal(ref_buf, got_buf, equal_nan=True)
    err = oracle.normwise_rel_err(logical_c(got_buf, c), oracle.sgemm(*oracle_args(c)))
    assert err <= BAR[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "T")])
def test_big_tile_equals_ordinary_call(prec, ta, tb):
    """3072 x 3072: 144 tiles of 256 x 256, the big packed tile."""
    c = synth.sgemm_case(52, ta, tb, 3072, 3072, 320, alpha=1.0, beta=0.0, pad=16)
    log("packed B %s 3072^2 x 320 %s%s" % (prec, ta, tb))
    ref_buf, got_buf = both(c, prec)
    assert np.array_equal(ref_buf, got_buf, equal_nan=True)


@pytest.mark.parametrize("prec", PRECS)
def test_one_handle_many_products(prec):
    """One packed B, three products with different A (M 500, 100, 1);
    each equals the ordinary call."""
    import torch
    K, N = 700, 300
    cb = synth.sgemm_case(53, "N", "N", 8, N, K, pad=5)
    B = to_dev(cb["B"])
    with mg.PackedB("N", K, N, B, cb["ldb"], precision=prec) as pb:
        info = pb.info()
        assert (info["K"], info["N"], info["precision"]) == (K, N, mg.PRECISIONS[prec])
        packed = ((N + 31) // 32) * ((K + 15) // 16) * 64 * 16 * (2 if prec == "bf16x3" else 1)
        assert info["bytes"] == packed if prec == "bf16x3" else info["bytes"] > packed
        for i, M in enumerate((500, 100, 1)):
            ca = synth.sgemm_case(60 + i, "T", "N", M, N, K, alpha=0.75, beta=0.25, pad=2)
            A, C1, C2 = to_dev(ca["A"]), to_dev(ca["C"]), to_dev(ca["C"])
            mg.sgemm("T", "N", M, N, K, 0.75, A, ca["lda"], B, cb["ldb"], 0.25, C1, ca["ldc"],
                     precision=prec, config=packed_config(M, N))
            pb.sgemm("T", M, 0.75, A, ca["lda"], 0.25, C2, ca["ldc"])
            torch.cuda.synchronize()
            log("packed B reuse M=%d" % M)
            assert torch.equal(C1, C2)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("K,alpha", [(0, 1.5), (40, 0.0)])
def test_no_product_scales_c(prec, K, alpha):
    """K = 0 (a handle with no packed data) or alpha = 0: C <- beta C."""
    import torch
    c = synth.sgemm_case(54, "N", "N", 50, 40, K, alpha=alpha, beta=-2.0, pad=2)
    B = to_dev(c["B"]) if c["B"].size else torch.empty(1, device="cuda")
    C = to_dev(c["C"])
    with mg.PackedB("N", K, 40, B, c["ldb"], precision=prec) as pb:
        pb.sgemm("N", 50, alpha, to_dev(c["A"]) if c["A"].size else None, c["lda"], -2.0, C,
                 c["ldc"])
    torch.cuda.synchronize()
    got = logical_c(C.cpu().numpy(), c)
    assert np.array_equal(got, -2.0 * logical_c(c["C"], c).astype(np.float64))


@pytest.mark.parametrize("prec", PRECS)
def test_wide_ldc(prec):
    """ldc above the 32-bit buffer path's limit: the packed kernel's 64-bit
    epilogue; equal to the ordinary call and within the form's bar."""
    c = wide_ldc_case(55, "T", "N", 300, 6, 200, alpha=1.5, beta=-0.5)
    log("packed B %s wide ldc" % prec)
    ref_buf, got_buf = both(c, prec)
    assert np.array_equal(ref_buf, got_buf, equal_nan=True)
    full_check(c, got_buf, bound_fn=None, normwise=BAR[prec])


# ---- FP32: op(B) transposed once ----------------------------------------------

def _op_b_as_n(c):
    """op(B) of the case as a stored K x N column-major array at ld K."""
    K, N, ldb = c["K"], c["N"], c["ldb"]
    if c["transB"] == "N":
        nk = c["B"].reshape(N, ldb)[:, :K]          # [n][k]
    else:
        nk = c["B"].reshape(K, ldb)[:, :N].T        # stored N x K: [k][n] -> [n][k]
    return np.ascontiguousarray(nk).reshape(-1).astype(np.float32)


@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("shape", [(300, 270, 77), (513, 257, 1000), (33, 65, 7), (1, 1, 1),
                                   (130, 70, 0), (1024, 768, 513)])
def test_fp32_packed_b_equals_n_operand_call_and_oracle(ta, tb, shape):
    import torch
    from gpu_util import fp32_bound
    M, N, K = shape
    c = synth.sgemm_case(54, ta, tb, M, N, K, alpha=1.5, beta=-0.5, pad=3)
    log("packed B fp32 %s %s%s" % (shape, ta, tb))
    A, B = to_dev(c["A"]), to_dev(c["B"])
    C1, C2 = to_dev(c["C"]), to_dev(c["C"])
    Bn = to_dev(_op_b_as_n(c)) if K > 0 else to_dev(np.zeros(1, np.float32))
    mg.sgemm(ta, "N", M, N, K, 1.5, A, c["lda"], Bn, max(1, K), -0.5, C1, c["ldc"])
    with mg.PackedB(tb, K, N, B, c["ldb"], precision="fp32") as pb:
        info = pb.info()
        assert info["precision"] == mg.PRECISIONS["fp32"]
        assert info["bytes"] == (((max(K, 1) + 3) // 4) * 4 * N * 4 if K > 0 and N > 0 else 0)
        pb.sgemm(ta, M, 1.5, A, c["lda"], -0.5, C2, c["ldc"])
    torch.cuda.synchronize()
    ref_buf, got_buf = C1.cpu().numpy(), C2.cpu().numpy()
    assert np.array_equal(ref_buf, got_buf, equal_nan=True)
    got = logical_c(got_buf, c)
    ref = oracle.sgemm(*oracle_args(c))
    assert np.all(np.abs(got - ref) <= fp32_bound(c) + 1e-30)


def test_fp32_one_handle_many_products_and_streams():
    """One FP32 packed B (stored 'T'), three products with different A on
    the current stream and on a side stream that waits for the pack."""
    import torch
    K, N = 600, 333
    cb = synth.sgemm_case(55, "N", "T", 8, N, K, pad=4)
    B = to_dev(cb["B"])
    side = torch.cuda.Stream()
    with mg.PackedB("T", K, N, B, cb["ldb"], precision="fp32") as pb:
        for i, (M, st) in enumerate(((400, None), (65, side), (1, None))):
            ca = synth.sgemm_case(70 + i, "T", "T", M, N, K, alpha=0.5, beta=0.25, pad=2)
            ca["B"], ca["ldb"] = cb["B"], cb["ldb"]
            A, C1, C2 = to_dev(ca["A"]), to_dev(ca["C"]), to_dev(ca["C"])
            mg.sgemm("T", "T", M, N, K, 0.5, A, ca["lda"], B, cb["ldb"], 0.25, C1, ca["ldc"])
            if st is not None:
                st.wait_stream(torch.cuda.current_stream())   # A and C2 are copied in
            pb.sgemm("T", M, 0.5, A, ca["lda"], 0.25, C2, ca["ldc"], stream=st)
            torch.cuda.synchronize()
            ref = oracle.sgemm(*oracle_args(ca))
            err = oracle.normwise_rel_err(logical_c(C2.cpu().numpy(), ca), ref)
            assert err <= 1e-6, (M, err)

