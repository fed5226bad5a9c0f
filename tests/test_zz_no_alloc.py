"""The entry point that allocates nothing: bx_radical_segment_dev_noalloc.

It is bx_radical_segment_dev with every scratch buffer taken from the library's
fixed device array.  Called through the C-ABI, it must give exactly the radicals
of bx_radical_segment_dev on two calls in a row (the second smaller, so that any
stale scratch contents of the first would show), write nothing past hi - lo,
leave the device's free memory unchanged, and refuse a segment length its
scratch cannot hold.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2506_01099_amd import Benelux, _lib

pytestmark = pytest.mark.gpu

SENTINEL = 0x5A5A5A5A5A5A5A5A
MARGIN = 4096


def _noalloc(ctx, lo, hi, out, stream):
    return _lib.load().bx_radical_segment_dev_noalloc(ctx._h, int(lo), int(hi), ctypes.c_void_p(out.data_ptr()),
                                                        ctypes.c_void_p(int(stream.cuda_stream)))


def test_noalloc_equals_radical_segment_dev():
    import torch

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    # The second range is smaller than the first and lies elsewhere.
    cases = [((1 << 36) - 3_000_000, (1 << 36) + 1_700_003), (12_345, 12_345 + 700_001)]
    with Benelux(device=0) as ctx:
        outs = [torch.full((hi - lo + MARGIN,), SENTINEL, dtype=torch.int64, device=dev) for lo, hi in cases]
        refs = [torch.empty(hi - lo, dtype=torch.int64, device=dev) for lo, hi in cases]
        warm = torch.empty(64, dtype=torch.int64, device=dev)
        # One small call first: the HIP runtime's own lazy set-up is not the library's.
        assert _noalloc(ctx, 2, 66, warm, stream) == 0, _lib.load().bx_last_error()
        torch.cuda.synchronize()
        free_before = torch.cuda.mem_get_info(dev)[0]
        for (lo, hi), out in zip(cases, outs):
            rc = _noalloc(ctx, lo, hi, out, stream)
            assert rc == 0, _lib.load().bx_last_error()
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info(dev)[0] == free_before
        for (lo, hi), ref in zip(cases, refs):
            ctx.radical_segment_dev(lo, hi, ref, stream)
        torch.cuda.synchronize()
        for (lo, hi), out, ref in zip(cases, outs, refs):
            n = hi - lo
            got = out.cpu().numpy()
            assert np.array_equal(got[:n], ref.cpu().numpy()), (lo, hi)
            assert np.all(got[n:] == SENTINEL), (lo, hi)
            head = oracle.radicals(lo, lo + 3000).astype(np.int64)
            assert np.array_equal(got[:3000], head), (lo, hi)
        assert np.array_equal(warm.cpu().numpy(), oracle.radicals(2, 66).astype(np.int64))


def test_noalloc_refuses_what_its_scratch_cannot_hold():
    import torch

    dev = torch.device("cuda", 0)
    with Benelux(device=0) as ctx:
        ctx.set_option("seg_len", 1 << 22)
        out = torch.full((1000,), SENTINEL, dtype=torch.int64, device=dev)
        rc = _noalloc(ctx, 1 << 40, (1 << 40) + 1000, out, torch.cuda.current_stream(dev))
        assert rc == _lib.BX_ENOMEM
        assert b"scratch" in _lib.load().bx_last_error()
        torch.cuda.synchronize()
        assert torch.all(out == SENTINEL)
        # Back at a segment length it can hold, the same context answers.
        ctx.set_option("seg_len", 0)
        assert _noalloc(ctx, 1 << 40, (1 << 40) + 1000, out, torch.cuda.current_stream(dev)) == 0
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.radicals(1 << 40, (1 << 40) + 1000).astype(np.int64))
