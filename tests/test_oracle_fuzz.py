"""The oracle's decoder under corrupted streams, built with address and
undefined-behaviour sanitizers (gcc): bit flips, byte stomps, every
truncation and garbage bodies all end in OK or ECORRUPT with no access
outside the exact buffers given."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_decoder_fuzz_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_fuzz")
    subprocess.run(["gcc", "-O1", "-std=c11", "-Wall", "-Werror", "-ffp-contract=off", "-fno-fast-math",
                    "-msse2", "-mfpmath=sse", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-D_DEFAULT_SOURCE", "-I", ORACLE, "-o", exe, os.path.join(HERE, "cpp", "oracle_fuzz.c"),
                    os.path.join(ORACLE, "szref.c"), "-lm"], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-3000:]
    assert "oracle fuzz ok" in out.stdout
