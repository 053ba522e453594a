"""Diagnostics switched on from the environment: MGEMM_LOG (one line per
call) and MGEMM_FAULT=alloc (every workspace, packed-operand or plan
allocation fails before anything is launched)."""
import ctypes

import numpy as np
import pytest

import paper_1912_04379_amd as mg
import synth
from paper_1912_04379_amd import _lib

FA, FB, FC = 0x10000000, 0x20000000, 0x30000000


def _ex(transA="N", transB="N", M=4, N=4, K=4, alpha=1.0, A=FA, lda=4, B=FB, ldb=4,
        beta=0.0, C=FC, ldc=4, precision=0, config=-1, stream=None):
    return mg.lib().mgemm_sgemm_ex(transA.encode(), transB.encode(), M, N, K, alpha, A, lda, B,
                                   ldb, beta, C, ldc, stream, precision, config)


def test_log_records_a_rejected_call(tmp_path, monkeypatch):
    log = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(log))
    assert _ex(transA="T", M=5, N=3, K=7, lda=6, precision=1) == -8
    line = log.read_text().strip().splitlines()[-1]
    assert line.startswith("mgemm: sgemm bf16x3 TN M=5 N=3 K=7 lda=6 ldb=4 ldc=4")
    assert "status=-8 lda < max(1, stored rows of A)" in line


def test_log_is_off_unless_asked(tmp_path, monkeypatch):
    log = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", "0")
    assert _ex(lda=3) == -8
    monkeypatch.delenv("MGEMM_LOG")
    assert _ex(lda=3) == -8
    assert not log.exists()


def test_log_records_quick_returns(tmp_path, monkeypatch):
    log = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(log))
    assert _ex(M=0, C=None, lda=1, ldc=1) == 0
    assert "-> none cfg=-1 splits=0 workspace=0 status=0" in log.read_text()


# ---- on the GPU ---------------------------------------------------------------

def _dev(buf):
    import torch
    return torch.from_numpy(np.ascontiguousarray(buf)).cuda()


@pytest.mark.gpu
def test_fault_alloc_fails_before_launching(monkeypatch):
    """With MGEMM_FAULT=alloc, every call that needs a workspace returns
    MGEMM_ERR_ALLOC and leaves C as it was; calls that need none still run;
    without it the same calls succeed."""
    import torch
    print("MGEMM_FAULT=alloc", flush=True)
    c = synth.sgemm_case(5, "N", "N", 300, 200, 4096, alpha=1.5, beta=-0.5)
    A, B, C = _dev(c["A"]), _dev(c["B"]), _dev(c["C"])
    s = torch.cuda.current_stream().cuda_stream

    def call(prec, cfg):
        return _ex("N", "N", 300, 200, 4096, 1.5, A.data_ptr(), c["lda"], B.data_ptr(), c["ldb"],
                   -0.5, C.data_ptr(), c["ldc"], precision=prec, config=cfg, stream=s)
    # Workspace-taking cases: FP32 and 16-bit split-K (this product's
    # default for both 16-bit forms), packed BF16x3 configurations, and the
    # FP16 exponents of every FP16 configuration.
    assert mg.lib().mgemm_default_config(1, b"N", b"N", 300, 200, 4096) == 13
    monkeypatch.setenv("MGEMM_FAULT", "alloc")
    for prec, cfg in ((0, 11), (1, -1), (1, 4), (1, 11), (1, 13), (2, 0), (2, -1)):
        assert call(prec, cfg) == _lib.ERR_ALLOC, (prec, cfg)
        assert b"workspace" in mg.lib().mgemm_last_error()
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), c["C"])
    pb = ctypes.c_void_p()
    assert mg.lib().mgemm_pack_b(b"N", 4096, 200, B.data_ptr(), c["ldb"], 1, s,
                                 ctypes.byref(pb)) == _lib.ERR_ALLOC
    assert not pb.value
    from paper_1912_04379_amd import grouped as gp
    probs = [dict(transA="N", transB="N", M=300, N=200, K=4096, alpha=1.5, beta=-0.5,
                  A=A.data_ptr(), lda=c["lda"], B=B.data_ptr(), ldb=c["ldb"], C=C.data_ptr(),
                  ldc=c["ldc"])]
    plan, bad = ctypes.c_void_p(), ctypes.c_int64()
    st = mg.lib().mgemm_grouped_plan_create(gp._problem_array(probs), 1, 0, None, None,
                                            ctypes.byref(plan), ctypes.byref(bad))
    assert st == _lib.ERR_ALLOC and not plan.value
    assert call(0, 0) == 0          # FP32 configuration 0 takes no workspace
    assert call(1, 3) == 0          # nor does BF16x3 split while staging
    monkeypatch.delenv("MGEMM_FAULT")
    for prec, cfg in ((0, 11), (1, -1), (1, 4), (2, -1)):
        assert call(prec, cfg) == 0
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_log_records_the_path_taken(tmp_path, monkeypatch):
    import torch
    print("MGEMM_LOG dispatch", flush=True)
    log = tmp_path / "mgemm.log"
    monkeypatch.setenv("MGEMM_LOG", str(log))
    c = synth.sgemm_case(6, "T", "N", 512, 512, 16384, alpha=1.0, beta=0.0)
    A, B, C = _dev(c["A"]), _dev(c["B"]), _dev(c["C"])
    s = torch.cuda.current_stream().cuda_stream
    for prec in (0, 1, 2):
        assert _ex("T", "N", 512, 512, 16384, 1.0, A.data_ptr(), c["lda"], B.data_ptr(),
                   c["ldb"], 0.0, C.data_ptr(), c["ldc"], precision=prec, stream=s) == 0
    torch.cuda.synchronize()
    lines = log.read_text().strip().splitlines()
    assert len(lines) == 3
    assert "sgemm fp32 TN M=512 N=512 K=16384" in lines[0]
    assert "-> f32_split_k cfg=11 splits=" in lines[0] and lines[0].endswith("status=0")
    assert "sgemm bf16x3" in lines[1] and "status=0" in lines[1]
    assert "sgemm fp16s" in lines[2] and "workspace=" in lines[2]
