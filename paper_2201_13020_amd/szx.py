"""Python binding of the C ABI in include/szx.h (argument marshalling only).

PyTorch provides device memory and streams; every step of compression and
decompression runs in the HIP kernels of ``libszx.so``. There is no fallback:
if the library or a GPU is missing, these functions raise.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libszx.so")

SZ_F32, SZ_F64 = 0, 1
SZ_ABS, SZ_REL = 0, 1
STATUS = {0: "SZ_OK", 1: "SZ_EINVAL", 2: "SZ_ENOSPC", 3: "SZ_ECORRUPT", 4: "SZ_EDEVICE",
          5: "SZ_ENOMEM", 6: "SZ_EUNSUPPORTED", 7: "SZ_EIO"}
HEADER_BYTES = 96


class SzParams(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_uint32),
        ("ndims", ctypes.c_uint32),
        ("dims", ctypes.c_uint64 * 4),
        ("eb_mode", ctypes.c_uint32),
        ("block_size", ctypes.c_uint32),
        ("eb", ctypes.c_double),
    ]


class SzCField(ctypes.Structure):
    _fields_ = [("params", SzParams), ("d_in", ctypes.c_void_p), ("d_out", ctypes.c_void_p),
                ("out_cap", ctypes.c_uint64), ("d_out_size", ctypes.c_void_p)]


class SzDField(ctypes.Structure):
    _fields_ = [("expected", SzParams), ("d_in", ctypes.c_void_p), ("in_bytes", ctypes.c_uint64),
                ("d_out", ctypes.c_void_p), ("out_cap", ctypes.c_uint64), ("d_status", ctypes.c_void_p)]


class SzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded libszx.so. Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(SzParams)
        vp, u64 = ctypes.c_void_p, ctypes.c_uint64
        L.sz_compress_bound.argtypes = [P]
        L.sz_compress_bound.restype = u64
        L.sz_workspace_size.argtypes = [P]
        L.sz_workspace_size.restype = u64
        L.sz_compress.argtypes = [P, vp, vp, u64, vp, vp, u64, vp]
        L.sz_compress.restype = ctypes.c_int
        L.sz_compress_noalloc.argtypes = [P, vp, vp, u64, vp, vp]
        L.sz_compress_noalloc.restype = ctypes.c_int
        L.sz_shard_params.argtypes = [P, u64, u64, P]
        L.sz_shard_params.restype = ctypes.c_int
        L.sz_range.argtypes = [P, vp, vp, vp, u64, vp]
        L.sz_range.restype = ctypes.c_int
        L.sz_compress_shard.argtypes = [P, u64, u64, vp, vp, ctypes.c_uint32, vp, u64, vp, vp, u64, vp]
        L.sz_compress_shard.restype = ctypes.c_int
        L.sz_stitch.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(vp), ctypes.POINTER(u64), vp, u64, vp, vp]
        L.sz_stitch.restype = ctypes.c_int
        L.sz_decompress.argtypes = [vp, u64, P, vp, u64, vp, vp, u64, vp]
        L.sz_decompress.restype = ctypes.c_int
        L.sz_inspect.argtypes = [vp, u64, P, ctypes.POINTER(u64)]
        L.sz_inspect.restype = ctypes.c_int
        L.sz_last_error.argtypes = []
        L.sz_last_error.restype = ctypes.c_char_p
        L.sz_timing_enable.argtypes = [ctypes.c_int]
        L.sz_timing_enable.restype = None
        L.sz_timing_read.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32]
        L.sz_timing_read.restype = ctypes.c_uint32
        CF, DF = ctypes.POINTER(SzCField), ctypes.POINTER(SzDField)
        L.sz_batch_workspace_size.argtypes = [CF, DF, ctypes.c_uint32]
        L.sz_batch_workspace_size.restype = u64
        L.sz_batch_create_compress.argtypes = [CF, ctypes.c_uint32, vp, u64, ctypes.POINTER(vp)]
        L.sz_batch_create_compress.restype = ctypes.c_int
        L.sz_batch_create_decompress.argtypes = [DF, ctypes.c_uint32, vp, u64, ctypes.POINTER(vp)]
        L.sz_batch_create_decompress.restype = ctypes.c_int
        L.sz_batch_set_geometry.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32]
        L.sz_batch_set_geometry.restype = ctypes.c_int
        L.sz_size_class.argtypes = [u64]
        L.sz_size_class.restype = ctypes.c_uint32
        L.sz_set_geometry.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.sz_set_geometry.restype = ctypes.c_int
        L.sz_batch_run.argtypes = [vp, vp]
        L.sz_batch_run.restype = ctypes.c_int
        L.sz_batch_destroy.argtypes = [vp]
        L.sz_batch_destroy.restype = None
        L.sz_file_write.argtypes = [ctypes.c_char_p, vp, u64, ctypes.c_int, vp]
        L.sz_file_write.restype = ctypes.c_int
        L.sz_file_size.argtypes = [ctypes.c_char_p, ctypes.POINTER(u64)]
        L.sz_file_size.restype = ctypes.c_int
        L.sz_file_read.argtypes = [ctypes.c_char_p, vp, u64, ctypes.POINTER(u64), vp]
        L.sz_file_read.restype = ctypes.c_int
        _lib = L
    return _lib


def _dtype_code(dtype):
    if dtype in (torch.float32, "float32", "f32", SZ_F32):
        return SZ_F32
    if dtype in (torch.float64, "float64", "f64", SZ_F64):
        return SZ_F64
    raise ValueError(f"unsupported dtype {dtype}")


def size_class(nbytes):
    return int(lib().sz_size_class(int(nbytes)))


def set_geometry(dtype, size_class, encode_wgs):
    """Process-wide encode geometry for one element type and size class
    (0 restores the default)."""
    _check(lib().sz_set_geometry(_dtype_code(dtype), int(size_class), int(encode_wgs)), "sz_set_geometry")


def _check(rc, what):
    if rc != 0:
        raise SzError(rc, f"{what}: {lib().sz_last_error().decode()}")


def make_params(dtype, dims, eb=0.0, mode="rel", block=128):
    p = SzParams()
    dt = torch.float32 if dtype in (torch.float32, "float32", "f32") else dtype
    if dt == torch.float32:
        p.dtype = SZ_F32
    elif dt in (torch.float64, "float64", "f64"):
        p.dtype = SZ_F64
    else:
        raise ValueError(f"unsupported dtype {dtype}")
    dims = tuple(int(d) for d in dims)
    if not 1 <= len(dims) <= 4:
        raise ValueError("1 to 4 dims")
    p.ndims = len(dims)
    for i, d in enumerate(dims):
        p.dims[i] = d
    p.eb_mode = SZ_REL if mode == "rel" else SZ_ABS
    p.block_size = int(block)
    p.eb = float(eb)
    return p


def params_dict(p):
    return dict(dtype=torch.float32 if p.dtype == SZ_F32 else torch.float64,
                dims=tuple(int(p.dims[i]) for i in range(p.ndims)),
                mode="rel" if p.eb_mode == SZ_REL else "abs",
                block=int(p.block_size), eb=float(p.eb))


def compress_bound(dtype, dims, eb=0.0, mode="rel", block=128):
    return int(lib().sz_compress_bound(ctypes.byref(make_params(dtype, dims, eb, mode, block))))


def workspace_size(dtype, dims, eb=0.0, mode="rel", block=128):
    return int(lib().sz_workspace_size(ctypes.byref(make_params(dtype, dims, eb, mode, block))))


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def compress(x, eb, mode="rel", block=128, dims=None, out=None, out_size=None, ws=None, stream=None):
    """Compress the device tensor x. Returns (out, out_size): the uint8 device
    buffer holding the stream and a 1-element uint64 device tensor with its
    size. Asynchronous on `stream` (default: torch's current stream)."""
    if not (x.is_cuda and x.is_contiguous() and x.dtype in (torch.float32, torch.float64)):
        raise ValueError("x must be a contiguous float32/float64 device tensor")
    dims = tuple(x.shape) if dims is None else tuple(dims)
    if len(dims) == 0:
        dims = (1,)
    p = make_params(x.dtype, dims, eb, mode, block)
    cap = int(lib().sz_compress_bound(ctypes.byref(p)))
    wsz = int(lib().sz_workspace_size(ctypes.byref(p)))
    if cap == 0 or wsz == 0:
        raise SzError(1, "invalid parameters: " + lib().sz_last_error().decode())
    # buffers made here belong to the stream the kernels run on, so that the
    # caching allocator does not hand them out again while that stream still
    # uses them
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream(x.device)):
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        if out_size is None:
            out_size = torch.empty(1, dtype=torch.uint64, device=x.device)
        if ws is None:
            ws = torch.empty(wsz, dtype=torch.uint8, device=x.device)
    rc = lib().sz_compress(ctypes.byref(p), _ptr(x), _ptr(out), out.numel(), _ptr(out_size),
                           _ptr(ws), ws.numel(), _stream_handle(stream))
    _check(rc, "sz_compress")
    return out, out_size


def compress_noalloc(x, eb, mode="rel", block=128, dims=None, out=None, out_size=None, stream=None):
    """sz_compress_noalloc: as compress(), with the library's static device
    scratch array as the workspace (no workspace tensor). Calls on one GPU
    share that array and must not overlap."""
    if not (x.is_cuda and x.is_contiguous() and x.dtype in (torch.float32, torch.float64)):
        raise ValueError("x must be a contiguous float32/float64 device tensor")
    dims = tuple(x.shape) if dims is None else tuple(dims)
    if len(dims) == 0:
        dims = (1,)
    p = make_params(x.dtype, dims, eb, mode, block)
    cap = int(lib().sz_compress_bound(ctypes.byref(p)))
    if cap == 0:
        raise SzError(1, "invalid parameters: " + lib().sz_last_error().decode())
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream(x.device)):
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=x.device)
        if out_size is None:
            out_size = torch.empty(1, dtype=torch.uint64, device=x.device)
    rc = lib().sz_compress_noalloc(ctypes.byref(p), _ptr(x), _ptr(out), out.numel(), _ptr(out_size),
                                   _stream_handle(stream))
    _check(rc, "sz_compress_noalloc")
    return out, out_size


# ------------------------------------------------------------------ shards --

def shard_params(field, k0, k1):
    """Parameters (SzParams) of the shard of blocks [k0, k1) of the field
    `field` (an SzParams) as a 1-D field."""
    out = SzParams()
    _check(lib().sz_shard_params(ctypes.byref(field), int(k0), int(k1), ctypes.byref(out)), "sz_shard_params")
    return out


def field_range(x, block=128, ws=None, out=None, stream=None):
    """Finite (min, max) of the device tensor x as a 2-element float64 device
    tensor ((+inf, -inf) when nothing is finite)."""
    p = make_params(x.dtype, (x.numel(),), 0.0, "rel", block)
    wsz = int(lib().sz_workspace_size(ctypes.byref(p)))
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream(x.device)):
        if ws is None:
            ws = torch.empty(max(wsz, 16), dtype=torch.uint8, device=x.device)
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=x.device)
    _check(lib().sz_range(ctypes.byref(p), _ptr(x), _ptr(out), _ptr(ws), ws.numel(), _stream_handle(stream)),
           "sz_range")
    return out


def compress_shard(field, k0, k1, x_shard, ranges, out=None, out_size=None, ws=None, stream=None):
    """sz_compress_shard: the stream of blocks [k0, k1) of the field `field`
    (SzParams), whose values are the device tensor x_shard, with the bound of
    the whole field from `ranges` (a float64 device tensor of (min, max)
    pairs). Returns (out, out_size) as compress() does."""
    sp = shard_params(field, k0, k1)
    if x_shard.numel() != sp.dims[0]:
        raise ValueError(f"shard holds {sp.dims[0]} values, got {x_shard.numel()}")
    cap = int(lib().sz_compress_bound(ctypes.byref(sp)))
    wsz = int(lib().sz_workspace_size(ctypes.byref(sp)))
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream(x_shard.device)):
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=x_shard.device)
        if out_size is None:
            out_size = torch.empty(1, dtype=torch.uint64, device=x_shard.device)
        if ws is None:
            ws = torch.empty(wsz, dtype=torch.uint8, device=x_shard.device)
    nr = 0 if ranges is None else ranges.numel() // 2
    rc = lib().sz_compress_shard(ctypes.byref(field), int(k0), int(k1), _ptr(x_shard), _ptr(ranges), nr, _ptr(out),
                                 out.numel(), _ptr(out_size), _ptr(ws), ws.numel(), _stream_handle(stream))
    _check(rc, "sz_compress_shard")
    return out, out_size


def stitch(field, shards, out=None, out_size=None, stream=None):
    """sz_stitch: the stream of the whole field `field` (SzParams) from its
    shard streams (uint8 device tensors, in block order). Returns (out,
    out_size)."""
    n = len(shards)
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in shards])
    caps = (ctypes.c_uint64 * n)(*[t.numel() for t in shards])
    cap = int(lib().sz_compress_bound(ctypes.byref(field)))
    dev = shards[0].device
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream(dev)):
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=dev)
        if out_size is None:
            out_size = torch.empty(1, dtype=torch.uint64, device=dev)
    rc = lib().sz_stitch(ctypes.byref(field), n, ptrs, caps, _ptr(out), out.numel(), _ptr(out_size),
                         _stream_handle(stream))
    _check(rc, "sz_stitch")
    return out, out_size


def inspect(header):
    """Parse a host copy of a stream header (bytes, numpy uint8 or CPU tensor)."""
    if isinstance(header, torch.Tensor):
        header = header.cpu().numpy().tobytes()
    elif not isinstance(header, (bytes, bytearray)):
        header = bytes(header)
    buf = ctypes.create_string_buffer(bytes(header), len(header))
    p = SzParams()
    total = ctypes.c_uint64()
    rc = lib().sz_inspect(ctypes.cast(buf, ctypes.c_void_p), len(header), ctypes.byref(p),
                          ctypes.byref(total))
    _check(rc, "sz_inspect")
    d = params_dict(p)
    d["total"] = int(total.value)
    return d


def decompress(data, nbytes, expected, out=None, status=None, ws=None, stream=None):
    """Decompress the stream in the uint8 device tensor `data` (nbytes bytes).
    `expected`: dict with dtype, dims, block (e.g. from inspect()). Returns
    (out, status): the values and a 1-element uint32 device tensor (0 = ok,
    3 = corrupt stream). Asynchronous on `stream`."""
    p = make_params(expected["dtype"], expected["dims"], expected.get("eb", 0.0),
                    expected.get("mode", "rel"), expected["block"])
    wsz = int(lib().sz_workspace_size(ctypes.byref(p)))
    if wsz == 0:
        raise SzError(1, "invalid parameters: " + lib().sz_last_error().decode())
    dt = torch.float32 if p.dtype == SZ_F32 else torch.float64
    n = 1
    for d in expected["dims"]:
        n *= int(d)
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream(data.device)):
        if out is None:
            out = torch.empty(n, dtype=dt, device=data.device)
        if status is None:
            status = torch.empty(1, dtype=torch.uint32, device=data.device)
        if ws is None:
            ws = torch.empty(wsz, dtype=torch.uint8, device=data.device)
    rc = lib().sz_decompress(_ptr(data), int(nbytes), ctypes.byref(p), _ptr(out), out.numel() * out.element_size(),
                             _ptr(status), _ptr(ws), ws.numel(), _stream_handle(stream))
    _check(rc, "sz_decompress")
    return out, status


def timing_enable(on=True):
    lib().sz_timing_enable(1 if on else 0)


def timing_read(cap=32):
    """{kernel name: (launches, total ms)} since the last read (synchronises)."""
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_uint32 * cap)()
    m = lib().sz_timing_read(names, ms, cnt, cap)
    return {names[i].decode(): (int(cnt[i]), float(ms[i])) for i in range(m)}


def to_host_stream(out, out_size):
    """Synchronise and return the compressed stream as bytes."""
    n = int(out_size.cpu().view(torch.int64).item())
    return out[:n].cpu().numpy().tobytes()


class Batch:
    """A planned batch: its descriptor table lives in `ws`; run() enqueues the
    passes over all fields (one launch per pass). Keeps the tensors it names
    alive for its own lifetime."""

    def __init__(self, handle, ws, keep, outs=None, sizes=None, statuses=None):
        self._h = handle
        self.ws = ws
        self._keep = keep
        self.outs = outs
        self.sizes = sizes
        self.statuses = statuses

    def run(self, stream=None):
        _check(lib().sz_batch_run(self._h, _stream_handle(stream)), "sz_batch_run")

    def set_geometry(self, encode_wgs, dtype=None):
        """Encode workgroups for the fields of one element type (both if None)."""
        for dt in ([SZ_F32, SZ_F64] if dtype is None else [_dtype_code(dtype)]):
            _check(lib().sz_batch_set_geometry(self._h, dt, int(encode_wgs)), "sz_batch_set_geometry")

    def close(self):
        if self._h:
            lib().sz_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compress_batch(xs, ebs, modes="rel", block=128, dims=None, outs=None, sizes=None, ws=None):
    """Plan a compression batch over the device tensors xs (mixed float32 and
    float64 allowed; one block size). Returns a Batch whose .outs[i] and
    .sizes[i] receive field i's stream and size on each run()."""
    n = len(xs)
    ebs = list(ebs) if hasattr(ebs, "__len__") else [ebs] * n
    modes = list(modes) if isinstance(modes, (list, tuple)) else [modes] * n
    dims = dims or [tuple(x.shape) if x.dim() else (1,) for x in xs]
    arr = (SzCField * n)()
    outs = outs or []
    sizes = sizes or []
    for i, x in enumerate(xs):
        if not (x.is_cuda and x.is_contiguous() and x.dtype in (torch.float32, torch.float64)):
            raise ValueError("batch inputs must be contiguous float32/float64 device tensors")
        p = make_params(x.dtype, dims[i], ebs[i], modes[i], block)
        cap = int(lib().sz_compress_bound(ctypes.byref(p)))
        if len(outs) <= i:
            outs.append(torch.empty(cap, dtype=torch.uint8, device=x.device))
        if len(sizes) <= i:
            sizes.append(torch.zeros(1, dtype=torch.uint64, device=x.device))
        arr[i].params = p
        arr[i].d_in = x.data_ptr()
        arr[i].d_out = outs[i].data_ptr()
        arr[i].out_cap = outs[i].numel()
        arr[i].d_out_size = sizes[i].data_ptr()
    wsz = int(lib().sz_batch_workspace_size(arr, None, n))
    if wsz == 0:
        raise SzError(1, "invalid batch: " + lib().sz_last_error().decode())
    if ws is None:
        ws = torch.empty(wsz, dtype=torch.uint8, device=xs[0].device)
    h = ctypes.c_void_p()
    _check(lib().sz_batch_create_compress(arr, n, _ptr(ws), ws.numel(), ctypes.byref(h)), "sz_batch_create_compress")
    return Batch(h, ws, (list(xs), arr), outs=outs, sizes=sizes)


def decompress_batch(streams, nbytes, expected, outs=None, statuses=None, ws=None):
    """Plan a decompression batch over device streams (uint8 tensors of
    nbytes[i] valid bytes) with per-field expected params (dicts as returned
    by inspect()). Returns a Batch with .outs[i] and .statuses[i]."""
    n = len(streams)
    arr = (SzDField * n)()
    outs = outs or []
    statuses = statuses or []
    for i, d in enumerate(streams):
        e = expected[i]
        p = make_params(e["dtype"], e["dims"], e.get("eb", 0.0), e.get("mode", "rel"), e["block"])
        cnt = 1
        for v in e["dims"]:
            cnt *= int(v)
        dt = torch.float32 if p.dtype == SZ_F32 else torch.float64
        if len(outs) <= i:
            outs.append(torch.empty(max(cnt, 1), dtype=dt, device=d.device))
        if len(statuses) <= i:
            statuses.append(torch.zeros(1, dtype=torch.uint32, device=d.device))
        arr[i].expected = p
        arr[i].d_in = d.data_ptr()
        arr[i].in_bytes = int(nbytes[i])
        arr[i].d_out = outs[i].data_ptr()
        arr[i].out_cap = outs[i].numel() * outs[i].element_size()
        arr[i].d_status = statuses[i].data_ptr()
    wsz = int(lib().sz_batch_workspace_size(None, arr, n))
    if wsz == 0:
        raise SzError(1, "invalid batch: " + lib().sz_last_error().decode())
    if ws is None:
        ws = torch.empty(wsz, dtype=torch.uint8, device=streams[0].device)
    h = ctypes.c_void_p()
    _check(lib().sz_batch_create_decompress(arr, n, _ptr(ws), ws.numel(), ctypes.byref(h)),
           "sz_batch_create_decompress")
    return Batch(h, ws, (list(streams), arr), outs=outs, statuses=statuses)


# ------------------------------------------------------------ stream files --

def file_write(path, data, nbytes=None, durable=False, stream=None):
    """Write the first nbytes bytes of the contiguous tensor `data` (device or
    host; default: all of it) to the file at path, once the work queued on
    `stream` (default: torch's current stream, for a device tensor) has
    finished. Blocks until the bytes are in the file; durable=True also
    flushes them to storage (fsync)."""
    if not data.is_contiguous():
        raise ValueError("data must be contiguous")
    total = data.numel() * data.element_size()
    n = total if nbytes is None else int(nbytes)
    if n < 0 or n > total:
        raise ValueError(f"nbytes {n} outside [0, {total}]")
    sh = _stream_handle(stream) if data.is_cuda else ctypes.c_void_p(None)
    _check(lib().sz_file_write(os.fsencode(path), _ptr(data) if total else None, n, 1 if durable else 0, sh),
           "sz_file_write")


def file_size(path):
    """Size in bytes of the file at path."""
    n = ctypes.c_uint64()
    _check(lib().sz_file_size(os.fsencode(path), ctypes.byref(n)), "sz_file_size")
    return int(n.value)


def file_read(path, out=None, device="cuda", stream=None):
    """Read the whole file at path into `out` (a contiguous tensor with room
    for it) or into a new uint8 tensor on `device`. The copies are complete on
    return. Returns (tensor, bytes read)."""
    if out is None:
        out = torch.empty(max(file_size(path), 1), dtype=torch.uint8, device=device)
    if not out.is_contiguous():
        raise ValueError("out must be contiguous")
    got = ctypes.c_uint64()
    sh = _stream_handle(stream) if out.is_cuda else ctypes.c_void_p(None)
    _check(lib().sz_file_read(os.fsencode(path), _ptr(out), out.numel() * out.element_size(), ctypes.byref(got), sh),
           "sz_file_read")
    return out, int(got.value)
