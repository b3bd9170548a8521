"""The benchmark's stream statistics and quality figures, checked on the CPU
against the stream reader and the brute-force ladder outcomes of the tests
(oracle streams; torch CPU tensors stand in for device ones)."""
import math

import numpy as np
import pytest
import torch

import bench
import ladder
import streamfmt as sf
from oracle import szref


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_stream_stats_counts_the_ladder_outcomes(dtype):
    x, eb = ladder.subnormal_field(dtype, 300, 128, 7)
    s = szref.compress(x, eb, "abs", 128)
    info = sf.parse(s)
    got = bench.stream_stats(torch.from_numpy(x), torch.from_numpy(s.copy()), None)
    want = ladder.outcomes_of_stream(x, info)
    assert got["ladder"]["first_rung"] == sum(1 for o, _ in want if o == "K0")
    assert got["ladder"]["second_rung_K0_plus_1"] == sum(1 for o, _ in want if o == "K0+1")
    assert got["ladder"]["raw_by_failure"] == sum(1 for o, _ in want if o == "raw")
    assert got["ladder"]["second_rung_K0_plus_1"] > 0 and got["ladder"]["raw_by_failure"] > 0
    n_nc = int(info["n_nc"])
    assert got["blocks"] == info["nblk"]
    assert math.isclose(got["constant_frac"] + got["coded_frac"] + got["raw_frac"], 1.0, abs_tol=1e-5)
    assert sum(got["K_hist"].values()) == n_nc
    for k, c in got["K_hist"].items():
        assert c == int(np.sum(info["K"] == k))


def test_stream_stats_codes_and_partial_last_block():
    from paper_2201_13020_amd import synth
    x = synth.sines_1d((1 << 14) + 77)
    s = szref.compress(x, 1e-4, "rel", 128)
    info = sf.parse(s)
    got = bench.stream_stats(torch.from_numpy(x), torch.from_numpy(s.copy()), None)
    want = np.zeros(4, dtype=np.int64)
    ranks = np.cumsum(info["state"]) - 1
    for k in np.nonzero(info["state"])[0]:
        r = ranks[k]
        if info["K"][r] == 0xFF:
            continue
        for c in sf.unpack_codes(info["codes"][r], sf.block_len(info, k)):
            want[c] += 1
    assert got["code_hist"] == want.tolist()
    assert got["raw_frac"] == 0.0
    assert got["ladder"]["second_rung_K0_plus_1"] == 0 and got["ladder"]["raw_by_failure"] == 0
    assert got["ladder"]["first_rung"] == int(info["n_nc"])


def test_quality_max_error_and_psnr():
    x = torch.linspace(-1, 3, 1000, dtype=torch.float64)
    y = x + 1e-3 * torch.sign(torch.sin(torch.arange(1000.0, dtype=torch.float64)))
    e_bits = int(np.float64(2e-3).view(np.uint64))
    q = bench.quality(x, y, e_bits, 8)
    d = (y - x).numpy()
    assert q["max_abs_err"] == pytest.approx(np.abs(d).max())
    assert q["max_err_over_e"] == pytest.approx(np.abs(d).max() / 2e-3)
    assert q["psnr_db"] == pytest.approx(20 * math.log10(4.0 / math.sqrt(np.mean(d * d))), abs=1e-3)


def test_all_cores_leg_runs_disjoint_slices():
    from paper_2201_13020_amd import synth
    x = synth.sines_1d(1 << 15)
    r = bench.cpu_all_cores(x, (1e-3,), seconds=0.05)
    assert r["cores"] == bench.host_cores() and r["value"] > 0
    assert bench.cpu_model()
