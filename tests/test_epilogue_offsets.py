"""Index arithmetic of the C epilogue of the buffer path, worked on the CPU
for the 512-problem grouped batch (every tile variant, every work-group,
wave, lane and accumulator register).

The epilogue writes the tile's 32 x 32 MFMA blocks through one buffer
descriptor rebased to the tile's first element of C, with a byte count of
4 * (stored extent of C - that first element), clamped to 0x7ffffff0.
Lane l of wave (wm, wn) holds, in register e of block (i, j), the element
m = wm + 32 i + l % 32, n = wn + 32 j + 8 (e / 4) + 4 (l / 32) + e % 4 of
the tile; its byte offset is 4 (m + n ldc) when m < M - m0 and n < N - n0,
else 0x80000000 (out of range, so the load reads 0 and the store is
dropped).

Checked here: every offset of an element inside C is below the
descriptor's byte count and fits 32 bits; every masked offset is at least
the byte count; the elements written cover C exactly once over a problem's
tiles.  The offsets do not depend on the order in which blocks are issued,
so the same holds for an epilogue that issues the loads of several blocks
before their stores.
"""
import numpy as np
import pytest

import synth

BUF_OOB = 0x80000000
BUF_MAX_RANGE = 0x7FFFFFF0

# Grouped tile variants: (BM, BN, waves along m, waves along n).
VARIANTS = {
    "fp32_64x64x16": (64, 64, 2, 2), "fp32_128x128x16": (128, 128, 2, 2),
    "fp32_64x64x32": (64, 64, 2, 2), "bf16x3_64x64": (64, 64, 2, 2),
    "bf16x3_128x128": (128, 128, 2, 2), "bf16x3_128x64": (128, 64, 2, 2),
}


def _lane_elements(BM, BN, WGM, WGN):
    """(m, n) relative to the tile origin for every (wave, block, lane,
    register) of the epilogue, in issue order."""
    WM, WN = BM // WGM, BN // WGN
    ms, ns = [], []
    lane = np.arange(64)
    e = np.arange(16)
    for wave in range(WGM * WGN):
        wm, wn = (wave % WGM) * WM, (wave // WGM) * WN
        for i in range(WM // 32):
            for j in range(WN // 32):
                m = wm + 32 * i + (lane % 32)[:, None] + 0 * e[None, :]
                n = wn + 32 * j + 8 * (e[None, :] // 4) + 4 * (lane // 32)[:, None] + e[None, :] % 4
                ms.append(m.ravel())
                ns.append(n.ravel())
    return np.concatenate(ms), np.concatenate(ns)


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_epilogue_offsets_in_range_for_the_grouped_batch(variant):
    BM, BN, WGM, WGN = VARIANTS[variant]
    tm_rel, tn_rel = _lane_elements(BM, BN, WGM, WGN)
    assert tm_rel.size == BM * BN
    for p in synth.grouped_problems(0, 512, 16, 512):
        M, N = p["M"], p["N"]
        ldc = M                                # the batch's tight leading dimension
        extent = (N - 1) * ldc + M
        written = np.zeros(M * N, dtype=np.int64)
        for tn in range(-(-N // BN)):
            for tm in range(-(-M // BM)):
                m0, n0 = tm * BM, tn * BN
                first = m0 + n0 * ldc
                nrec = min(4 * (extent - first), BUF_MAX_RANGE)
                inside = (tm_rel < M - m0) & (tn_rel < N - n0)
                raw = 4 * (tm_rel + tn_rel.astype(np.int64) * ldc)
                off = np.where(inside, raw, BUF_OOB)
                assert np.all(off[inside] < nrec), (variant, p, tm, tn)
                assert np.all(off[inside] < 2 ** 32)
                assert np.all(off[~inside] >= nrec)
                idx = first + raw[inside] // 4
                written += np.bincount(idx, minlength=M * N)[:M * N] if idx.size else 0
        assert np.all(written == 1), (variant, p)


def test_descriptor_range_never_clamped_in_the_batch():
    """The largest descriptor of the batch is far below the clamp, so the
    clamp never turns an in-range element into a masked one here."""
    worst = max(4 * ((p["N"] - 1) * p["M"] + p["M"]) for p in synth.grouped_problems(0, 512, 16, 512))
    assert worst < BUF_MAX_RANGE
