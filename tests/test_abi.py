"""The C-ABI library loads and exports every symbol include/szx.h declares;
host-only entry points behave as documented (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("szx.h", "szx_server.h", "szx_io.h")]


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
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


def test_size_classes_and_geometry_table():
    from paper_2201_13020_amd import szx
    K = 1 << 10
    cases = [(0, 0), (256 * K - 1, 0), (256 * K, 1), (1 << 20, 2), (4 << 20, 3), (16 << 20, 4),
             (64 << 20, 5), (256 << 20, 6), (1 << 30, 7), (1 << 40, 7)]
    for nbytes, c in cases:
        assert szx.size_class(nbytes) == c, nbytes
    szx.set_geometry("f32", 3, 512)
    szx.set_geometry("f32", 3, 0)  # back to the default
    with pytest.raises(szx.SzError):
        szx.set_geometry("f64", 8, 1)
    L = szx.lib()
    assert L.sz_batch_set_geometry(None, 0, 64) == 1  # SZ_EINVAL
    assert L.sz_batch_run(None, None) == 1


def test_batch_planning_errors_without_a_device():
    """Batch sizing is host-only: mixed block sizes, an empty batch, both or
    neither of the field kinds give 0."""
    from paper_2201_13020_amd import szx
    import torch
    L = szx.lib()
    arr = (szx.SzCField * 2)()
    arr[0].params = szx.make_params(torch.float32, (1000,), 1e-3, "rel", 128)
    arr[1].params = szx.make_params(torch.float64, (77, 3), 1e-3, "abs", 128)
    one = int(L.sz_batch_workspace_size(arr, None, 2))
    assert one > 0
    assert L.sz_batch_workspace_size(arr, None, 0) == 0
    darr = (szx.SzDField * 1)()
    darr[0].expected = arr[0].params
    assert L.sz_batch_workspace_size(arr, darr, 1) == 0
    assert L.sz_batch_workspace_size(None, None, 1) == 0
    assert L.sz_batch_workspace_size(None, darr, 1) > 0
    arr[1].params = szx.make_params(torch.float64, (77, 3), 1e-3, "abs", 64)
    assert L.sz_batch_workspace_size(arr, None, 2) == 0


def test_server_entry_points_fail_cleanly_without_a_device():
    """Creating a server needs a device; without one the error comes back as
    SZ_EDEVICE and the other entry points reject a null server."""
    from paper_2201_13020_amd import serve, szx
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(szx.SzError) as e:
        serve.Server(hbm_budget=1 << 30)
    assert e.value.code == 4
    L = serve._lib()
    rid = ctypes.c_uint64()
    p = szx.make_params(torch.float32, (100,), 1e-3, "rel", 128)
    assert L.sz_server_submit_compress(None, ctypes.byref(p), None, 0, ctypes.byref(rid)) == 1
    assert L.sz_server_poll(None, None, 0, 0) == 0
    assert L.sz_server_release(None, 1) == 1
    cfg = serve.SzServerConfig(device=0, hbm_budget=1 << 30, slots=0, max_batch=1, block_size=128)
    h = ctypes.c_void_p()
    assert L.sz_server_create(ctypes.byref(cfg), ctypes.byref(h)) == 1  # slots out of range


def test_noalloc_size_limit_is_decided_on_the_host():
    """sz_compress_noalloc rejects a field whose workspace exceeds its static
    scratch array before any device call (so this runs without a GPU)."""
    import torch
    from paper_2201_13020_amd import szx
    L = szx.lib()
    dims = (1 << 31,)
    assert szx.workspace_size(torch.float32, dims, 1e-3, "rel", 128) > (32 << 20)
    p = szx.make_params("float32", dims, 1e-3, "rel", 128)
    assert L.sz_compress_noalloc(ctypes.byref(p), None, None, 0, None, None) == 6  # SZ_EUNSUPPORTED
    assert b"scratch" in L.sz_last_error()
    p.block_size = 12
    assert L.sz_compress_noalloc(ctypes.byref(p), None, None, 0, None, None) == 1  # SZ_EINVAL


def test_shard_params_and_their_checks():
    """Shard block ranges are checked on the host: multiples of 8 blocks
    (the field's end excepted), inside the field."""
    from paper_2201_13020_amd import szx
    field = szx.make_params("float32", (10, 1000), 1e-3, "rel", 128)  # 79 blocks, last one short
    sp = szx.shard_params(field, 8, 24)
    assert sp.ndims == 1 and sp.dims[0] == 16 * 128 and sp.block_size == 128 and sp.eb_mode == field.eb_mode
    sp = szx.shard_params(field, 72, 79)
    assert sp.dims[0] == 10000 - 72 * 128
    for k0, k1 in [(4, 24), (8, 20), (8, 80), (8, 8), (16, 8)]:
        with pytest.raises(szx.SzError):
            szx.shard_params(field, k0, k1)
