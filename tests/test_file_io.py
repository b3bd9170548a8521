"""Stream files (include/szx_io.h): the error paths and the empty file, which
touch no device (the round trips through device memory are in
test_gpu_io.py)."""
import os

import pytest

torch = pytest.importorskip("torch")


def _szx():
    from paper_2201_13020_amd import szx
    return szx


def test_write_into_a_missing_directory_is_an_io_error(tmp_path):
    szx = _szx()
    with pytest.raises(szx.SzError) as e:
        szx.file_write(str(tmp_path / "no" / "such" / "dir" / "s.szx"), torch.zeros(0, dtype=torch.uint8))
    assert e.value.code == 7 and "cannot create" in str(e.value)


def test_size_and_read_of_missing_or_odd_paths(tmp_path):
    szx = _szx()
    for f in (lambda: szx.file_size(str(tmp_path / "missing")),
              lambda: szx.file_size(str(tmp_path)),  # a directory
              lambda: szx.file_read(str(tmp_path / "missing"), out=torch.empty(4, dtype=torch.uint8))):
        with pytest.raises(szx.SzError) as e:
            f()
        assert e.value.code == 7


def test_null_arguments_are_rejected():
    szx = _szx()
    L = szx.lib()
    import ctypes
    n = ctypes.c_uint64()
    assert L.sz_file_write(None, None, 0, 0, None) == 1
    assert L.sz_file_write(b"/tmp/x", None, 5, 0, None) == 1
    assert L.sz_file_size(None, ctypes.byref(n)) == 1
    assert L.sz_file_read(b"/tmp/x", None, 0, ctypes.byref(n), None) == 1


def test_file_larger_than_the_destination(tmp_path):
    szx = _szx()
    p = tmp_path / "ten"
    p.write_bytes(bytes(range(10)))
    assert szx.file_size(str(p)) == 10
    with pytest.raises(szx.SzError) as e:
        szx.file_read(str(p), out=torch.empty(4, dtype=torch.uint8))
    assert e.value.code == 2  # SZ_ENOSPC, before any copy


def test_empty_file_round_trip(tmp_path):
    szx = _szx()
    p = str(tmp_path / "empty")
    with open(p, "wb") as f:
        f.write(b"junk")  # truncated by the write
    szx.file_write(p, torch.zeros(0, dtype=torch.uint8))
    assert os.path.getsize(p) == 0 and szx.file_size(p) == 0
    out, n = szx.file_read(p, out=torch.empty(1, dtype=torch.uint8))
    assert n == 0
