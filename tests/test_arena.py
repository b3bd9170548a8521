"""The serving runtime's device-arena allocator (host bookkeeping, no GPU):
built with g++ and run under address and undefined-behaviour sanitizers."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_allocator(tmp_path):
    exe = str(tmp_path / "arena_test")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-o", exe, os.path.join(HERE, "cpp", "arena_test.cpp")], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=120)
    assert "arena ok" in out.stdout
