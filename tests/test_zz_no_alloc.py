"""lv_encode_noalloc (the storage codec with its per-channel absmax scratch in
a static device array) against lv_encode, through the C ABI: identical codes
and scales on two calls in a row, the second smaller; no device allocation
during the call (a counting allocator is registered); sizes beyond the
static scratch are rejected."""
import gc

import numpy as np
import pytest
import torch

import paper_2410_14462_amd as lv
from synth import philox

pytestmark = pytest.mark.gpu


def call(fn, src, dtype, dst, scales):
    """One call of lv_encode or lv_encode_noalloc through the C ABI."""
    D = src.shape[-1]
    return getattr(lv.lib(), fn)(src.data_ptr(), src.numel() // D, D, dtype, dst.data_ptr(),
                                 scales.data_ptr() if scales is not None else None,
                                 torch.cuda.current_stream().cuda_stream)


def test_noalloc_encode_equals_encode_and_allocates_nothing():
    gc.collect()
    torch.cuda.synchronize()
    lv.release_scratch()
    assert lv.memory_stats() == (0, 0)
    counts = {"alloc": 0}

    def alloc(nbytes, stream):
        counts["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(max(nbytes, 1), 0, stream or 0)

    def free(ptr, nbytes, stream):
        torch.cuda.caching_allocator_delete(ptr)

    lv.set_allocator(alloc, free)
    try:
        for k, (H, W, D) in enumerate(((96, 120, 384), (40, 33, 24))):  # second call smaller
            src = torch.as_tensor(philox.normal(300 + k, 0, H * W * D).reshape(H, W, D) *
                                  np.linspace(0.01, 50.0, D, dtype=np.float32), device="cuda")
            src[:, :, 3] = 0.0  # an all-zero channel (scale 1)
            for dt, tdt in ((lv.LV_FP8_E4M3, torch.uint8), (lv.LV_BF16, torch.bfloat16)):
                a = torch.empty((H, W, D), device="cuda", dtype=tdt)
                b = torch.full((H, W, D), 7, device="cuda", dtype=tdt)
                sa = torch.empty(D, device="cuda") if dt == lv.LV_FP8_E4M3 else None
                sb = torch.full((D,), -1.0, device="cuda") if dt == lv.LV_FP8_E4M3 else None
                torch.cuda.synchronize()
                n0 = counts["alloc"]
                assert call("lv_encode", src, dt, a, sa) == 0
                n1 = counts["alloc"]
                assert call("lv_encode_noalloc", src, dt, b, sb) == 0
                torch.cuda.synchronize()
                assert counts["alloc"] == n1, "lv_encode_noalloc allocated device memory"
                assert lv.memory_stats() == (0, 0)
                if dt == lv.LV_FP8_E4M3:
                    assert n1 > n0  # lv_encode takes its absmax scratch from the allocator
                    assert torch.equal(sa, sb) and float(sb[3]) == 1.0
                assert torch.equal(a.view(torch.uint8) if tdt == torch.uint8 else a.view(torch.int16),
                                   b.view(torch.uint8) if tdt == torch.uint8 else b.view(torch.int16)), (k, dt)
        big = torch.zeros((2, 2, 4097), device="cuda")
        assert call("lv_encode_noalloc", big, lv.LV_FP8_E4M3, torch.empty_like(big, dtype=torch.uint8),
                    torch.empty(4097, device="cuda")) == 1
        assert b"static scratch" in lv.lib().lv_last_error()
    finally:
        gc.collect()
        torch.cuda.synchronize()
        lv.release_scratch()
        lv.set_allocator(None)
