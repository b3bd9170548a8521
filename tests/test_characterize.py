"""The characterisation tools on the CPU, on oracle streams: eq. (6) counts
checked against the stream's own mid-byte total and a brute-force loop, and
the block-range CDF against closed forms."""
import numpy as np
import pytest
import torch

from oracle import szref
import streamfmt as sf


def _overhead_brute(x, info):
    """Per value, the unshifted stored bits K - 8 c0 summed over non-raw
    non-constant blocks, written as plain loops."""
    b, n, w = info["b"], info["n"], info["w"]
    W = 8 * w
    udt = info["udtype"]
    nc = np.nonzero(info["state"])[0]
    total = 0
    for r, k in enumerate(nc):
        K = int(info["K"][r])
        if K == 0xFF:
            continue
        mu = info["mu"][k]
        prev = 0
        for i in range(k * b, min(n, (k + 1) * b)):
            v = np.array([x[i] - mu], dtype=info["dtype"])  # fl(x - mu) in T
            q = int(v.view(udt)[0]) >> (W - K) << (W - K)
            d = q ^ prev
            lead = 0
            while lead < 3 and (d >> (W - 8 * (lead + 1))) & 0xFF == 0:
                lead += 1
            total += K - 8 * min(lead, K // 8)
            prev = q
    return total


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("block", [8, 16, 128])
def test_space_overhead_counts(dtype, block):
    from paper_2201_13020_amd import characterize, synth
    x = (synth.sines_1d(3001) * 10).astype(dtype)
    x[100:140] = np.nan  # a raw block or two, left out of both counts
    s = szref.compress(x, 1e-3, "rel", block)
    info = sf.parse(s)
    r = characterize.space_overhead(torch.from_numpy(x), torch.from_numpy(s.copy()), block)
    raw = sum(sf.block_len(info, k) * info["w"] for j, k in enumerate(np.nonzero(info["state"])[0])
              if info["K"][j] == 0xFF)
    assert r["bits_shifted"] == 8 * (info["mid_total"] - raw)
    assert r["bits_unshifted"] == _overhead_brute(x, info)
    assert r["overhead"] == pytest.approx((r["bits_shifted"] - r["bits_unshifted"]) / (8.0 * s.size), abs=1e-6)


def test_block_range_cdf_closed_forms():
    from paper_2201_13020_amd import characterize
    # a ramp 0..N-1: every full block of b has relative range (b-1)/(N-1)
    N = 4096
    x = torch.arange(N, dtype=torch.float64)
    out = characterize.block_range_cdf(x, blocks=(8, 64), thresholds=(7 / 4095, 63 / 4095 - 1e-12, 63 / 4095))
    assert out[8][7 / 4095] == 1.0
    assert out[64][63 / 4095 - 1e-12] == 0.0 and out[64][63 / 4095] == 1.0
    # a constant field: every block has range 0
    c = torch.full((1000,), 2.5)
    assert characterize.block_range_cdf(c, blocks=(8,), thresholds=(0.0,))[8][0.0] == 1.0
