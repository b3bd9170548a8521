"""Helpers of the GPU tests: run the HIP path through the C ABI."""
import numpy as np
import torch

from paper_2201_13020_amd import szx


def gpu_compress(x_np, eb, mode="rel", block=128, dims=None):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    out, size = szx.compress(x, eb, mode, block, dims=dims)
    torch.cuda.synchronize()
    n = int(size.cpu().view(torch.int64).item())
    return out, n


def gpu_roundtrip(x_np, eb, mode="rel", block=128, dims=None):
    """(stream bytes as uint8 numpy, decoded values numpy, device status)."""
    out, n = gpu_compress(x_np, eb, mode, block, dims)
    assert n > 0, "device reported a failed compression"
    stream = out[:n].cpu().numpy()
    info = szx.inspect(stream[:96].tobytes())
    y, st = szx.decompress(out, n, info)
    torch.cuda.synchronize()
    return stream, y.cpu().numpy().reshape(info["dims"]), int(st.cpu().view(torch.int32).item())


def gpu_decompress(stream_np, expected=None):
    s = np.ascontiguousarray(stream_np, dtype=np.uint8)
    info = expected or szx.inspect(s[:96].tobytes())
    d = torch.from_numpy(s.copy()).cuda()
    y, st = szx.decompress(d, s.size, info)
    torch.cuda.synchronize()
    return y.cpu().numpy(), int(st.cpu().view(torch.int32).item())


def same_bits(a, b):
    a = np.ascontiguousarray(a).ravel()
    b = np.ascontiguousarray(b).ravel()
    if a.dtype != b.dtype or a.size != b.size:
        return False
    u = np.uint32 if a.dtype == np.float32 else np.uint64
    return np.array_equal(a.view(u), b.view(u))


def first_diff(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    n = min(a.size, b.size)
    d = np.nonzero(a[:n] != b[:n])[0]
    return int(d[0]) if d.size else (n if a.size != b.size else -1)
