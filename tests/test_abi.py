"""The C-ABI library loads and exports every symbol include/szx.h declares;
host-only entry points behave as documented (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "szx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sz_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["sz_compress", "sz_decompress", "sz_compress_bound", "sz_workspace_size",
              "sz_inspect", "sz_last_error", "sz_timing_enable", "sz_timing_read"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2201_13020_amd import szx
    L = szx.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
    assert os.path.dirname(szx.LIB_PATH) == os.path.join(ROOT, "paper_2201_13020_amd")


def test_compress_bound_and_workspace():
    from paper_2201_13020_amd import szx
    from oracle import szref
    import torch
    for dt, npdt in [(torch.float32, np.float32), (torch.float64, np.float64)]:
        for dims in [(1,), (1000,), (100, 500, 500), (7, 3, 11, 13)]:
            for b in [8, 128, 1024]:
                a = szx.compress_bound(dt, dims, 1e-3, "rel", b)
                assert a == szref.compress_bound(npdt, dims, 1e-3, "rel", b)
                assert szx.workspace_size(dt, dims, 1e-3, "rel", b) > 0
    assert szx.compress_bound(torch.float32, (10,), 1e-3, "rel", 100) == 0
    assert szx.compress_bound(torch.float32, (10,), -1.0, "rel", 128) == 0


def test_inspect_matches_oracle_streams():
    from paper_2201_13020_amd import szx
    from oracle import szref
    x = np.linspace(0, 1, 5000, dtype=np.float32).reshape(50, 100)
    s = szref.compress(x, 1e-3, "rel", 64)
    d = szx.inspect(s[:96].tobytes())
    assert d["dims"] == (50, 100) and d["block"] == 64 and d["mode"] == "rel"
    assert d["total"] == len(s)
    bad = bytearray(s[:96].tobytes())
    bad[0] ^= 1
    with pytest.raises(szx.SzError):
        szx.inspect(bytes(bad))
    with pytest.raises(szx.SzError):
        szx.inspect(s[:50].tobytes())


def test_argument_errors_are_returned_without_a_device():
    from paper_2201_13020_amd import szx
    L = szx.lib()
    p = szx.make_params("float32", (100,), 1e-3, "rel", 128)
    # null buffers are rejected before any device call
    rc = L.sz_compress(ctypes.byref(p), None, None, 0, None, None, 0, None)
    assert rc == 1
    assert b"null" in L.sz_last_error()
    p.block_size = 12
    assert L.sz_compress(ctypes.byref(p), None, None, 0, None, None, 0, None) == 1
