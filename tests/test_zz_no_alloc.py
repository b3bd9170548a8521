"""sz_compress_noalloc, whose workspace is the library's static device array,
against sz_compress with a workspace of the caller's: identical stream bytes
and sizes on calls in a row on one GPU, each later call with a smaller input
than the one before, so that what an earlier call left in the shared array
must not leak into a later stream."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2201_13020_amd import synth, szx


def _stream_bytes(out, size):
    n = int(size.cpu().view(torch.int64).item())
    assert n > 0, "device reported a failed compression"
    return out[:n].cpu().numpy()


def _cases():
    # largest first; each later input is smaller, with a ragged last block
    yield "turbulence 100x500x500 float32, REL 1e-3", synth.turbulence_3d((100, 500, 500)), 1e-3, "rel", 128
    yield "sines 2^16 + 37 float32, REL 1e-2", synth.sines_1d((1 << 16) + 37), 1e-2, "rel", 128
    rng = np.random.default_rng(13020 + 7)
    x = np.cumsum(rng.standard_normal(5003)).astype(np.float64)
    yield "random walk 5003 float64, ABS 1e-3, block 64", x, 1e-3, "abs", 64


@pytest.mark.gpu
def test_noalloc_equals_workspace_call_on_shrinking_inputs():
    for name, x_np, eb, mode, block in _cases():
        print(f"[no-alloc] {name}", flush=True)
        x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
        out_a, size_a = szx.compress(x, eb, mode, block)
        out_b, size_b = szx.compress_noalloc(x, eb, mode, block)
        torch.cuda.synchronize()
        a = _stream_bytes(out_a, size_a)
        b = _stream_bytes(out_b, size_b)
        assert a.size == b.size, f"{name}: size {b.size} vs {a.size}"
        assert np.array_equal(a, b), f"{name}: first differing byte {int(np.nonzero(a != b)[0][0])}"


@pytest.mark.gpu
def test_noalloc_repeated_call_is_deterministic():
    x_np = synth.sines_1d(1 << 18)
    x = torch.from_numpy(x_np).cuda()
    first = None
    for _ in range(3):
        out, size = szx.compress_noalloc(x, 1e-3, "rel", 128)
        torch.cuda.synchronize()
        got = _stream_bytes(out, size)
        if first is None:
            first = got
        assert np.array_equal(got, first)


@pytest.mark.gpu
def test_noalloc_rejects_fields_beyond_the_scratch_array():
    L = szx.lib()
    p = szx.make_params("float32", (1 << 31,), 1e-3, "rel", 128)
    assert szx.workspace_size(torch.float32, (1 << 31,), 1e-3, "rel", 128) > (32 << 20)
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    out = torch.zeros(16, dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.uint64, device="cuda")
    rc = L.sz_compress_noalloc(ctypes.byref(p), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               out.numel(), ctypes.c_void_p(size.data_ptr()), None)
    assert rc == 6  # SZ_EUNSUPPORTED, nothing enqueued
    assert b"scratch" in L.sz_last_error()
