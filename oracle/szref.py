"""ctypes binding of the CPU oracle ``libszref.so`` (test infrastructure only).

Host numpy arrays in, host numpy arrays out. Only the tests, the smoke check and
the benchmark's CPU-baseline leg may use this module.
"""
import ctypes
import os

import numpy as np

from . import build as _build

F32, F64 = 0, 1
ABS, REL = 0, 1
OK, EINVAL, ENOSPC, ECORRUPT, ENOMEM = 0, 1, 2, 3, 5


class Params(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_uint32),
        ("ndims", ctypes.c_uint32),
        ("dims", ctypes.c_uint64 * 4),
        ("eb_mode", ctypes.c_uint32),
        ("block_size", ctypes.c_uint32),
        ("eb", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load the oracle library, building it first only if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.POINTER(Params)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.szref_compress_bound.argtypes = [P]
        L.szref_compress_bound.restype = ctypes.c_uint64
        L.szref_error_bound.argtypes = [P, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        L.szref_error_bound.restype = ctypes.c_int
        L.szref_compress.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, u64p]
        L.szref_compress.restype = ctypes.c_int
        L.szref_inspect.argtypes = [ctypes.c_void_p, ctypes.c_uint64, P, u64p]
        L.szref_inspect.restype = ctypes.c_int
        L.szref_decompress.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64]
        L.szref_decompress.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def make_params(x_dtype, dims, eb, mode="rel", block=128):
    p = Params()
    p.dtype = F32 if np.dtype(x_dtype) == np.float32 else F64
    dims = tuple(int(d) for d in dims)
    p.ndims = len(dims)
    for i, d in enumerate(dims):
        p.dims[i] = d
    p.eb_mode = REL if mode == "rel" else ABS
    p.block_size = int(block)
    p.eb = float(eb)
    return p


def _dims_of(x, dims):
    return tuple(x.shape) if dims is None else tuple(dims)


def compress_bound(dtype, dims, eb=0.0, mode="rel", block=128):
    return int(lib().szref_compress_bound(ctypes.byref(make_params(dtype, dims, eb, mode, block))))


def error_bound(x, eb, mode="rel", block=128, dims=None):
    x = np.ascontiguousarray(x)
    p = make_params(x.dtype, _dims_of(x, dims), eb, mode, block)
    out = ctypes.c_double()
    rc = lib().szref_error_bound(ctypes.byref(p), x.ctypes.data, ctypes.byref(out))
    if rc != OK:
        raise OracleError(rc, "error_bound")
    return out.value


def compress(x, eb, mode="rel", block=128, dims=None):
    """Compress a float32/float64 array; returns the stream as a uint8 array."""
    x = np.ascontiguousarray(x)
    assert x.dtype in (np.float32, np.float64)
    p = make_params(x.dtype, _dims_of(x, dims), eb, mode, block)
    cap = int(lib().szref_compress_bound(ctypes.byref(p)))
    if cap == 0:
        raise OracleError(EINVAL, "compress_bound")
    out = np.zeros(cap, dtype=np.uint8)
    size = ctypes.c_uint64()
    rc = lib().szref_compress(ctypes.byref(p), x.ctypes.data if x.size else None,
                              out.ctypes.data, cap, ctypes.byref(size))
    if rc != OK:
        raise OracleError(rc, "compress")
    return out[: size.value].copy()


def inspect(stream):
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    p = Params()
    total = ctypes.c_uint64()
    rc = lib().szref_inspect(s.ctypes.data, s.size, ctypes.byref(p), ctypes.byref(total))
    if rc != OK:
        raise OracleError(rc, "inspect")
    dims = tuple(int(p.dims[i]) for i in range(p.ndims))
    return {
        "dtype": np.float32 if p.dtype == F32 else np.float64,
        "dims": dims,
        "eb_mode": "rel" if p.eb_mode == REL else "abs",
        "block": int(p.block_size),
        "eb": float(p.eb),
        "total": int(total.value),
    }


def decompress(stream):
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    info = inspect(s)
    n = int(np.prod(info["dims"], dtype=np.int64))
    out = np.empty(n, dtype=info["dtype"])
    rc = lib().szref_decompress(s.ctypes.data, s.size, out.ctypes.data if n else None,
                                out.nbytes)
    if rc != OK:
        raise OracleError(rc, "decompress")
    return out.reshape(info["dims"])


def decompress_status(stream):
    """Decoder status code for a (possibly corrupt) stream, without raising."""
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    try:
        info = inspect(s)
    except OracleError as err:
        return err.code
    n = int(np.prod(info["dims"], dtype=np.int64))
    out = np.empty(max(n, 1), dtype=info["dtype"])
    return int(lib().szref_decompress(s.ctypes.data, s.size, out.ctypes.data, out.nbytes))
