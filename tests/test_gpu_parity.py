"""Parity of the HIP path with the CPU oracle, through the C ABI.

Compressed streams must equal the oracle's byte for byte; decompressed values
must equal the oracle's bit for bit. Cases span several tiles with ragged
tails, every block size, both element types, both bound modes, and the
degenerate inputs of the method (empty, constant, raw, zero bound).
"""
import json
import os

import numpy as np
import pytest

from oracle import szref
import streamfmt as sf
from gpu_util import first_diff, gpu_compress, gpu_decompress, gpu_roundtrip, same_bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_13020_amd import szx
    szx.lib()  # fails loudly if the HIP library is missing


def check_parity(x, eb, mode="rel", block=128, label=""):
    print(f"[parity] {label} n={x.size} dtype={x.dtype} eb={eb} mode={mode} b={block}", flush=True)
    ref = szref.compress(x, eb, mode, block)
    stream, y, st = gpu_roundtrip(x, eb, mode, block)
    assert st == 0
    assert stream.size == ref.size, f"size {stream.size} vs oracle {ref.size}"
    assert np.array_equal(stream, ref), f"first differing byte {first_diff(stream, ref)}"
    yref = szref.decompress(ref)
    assert same_bits(y, yref), f"first differing value {first_diff(y.view(np.uint8), yref.view(np.uint8))}"
    return ref


def smooth(n, seed, dtype=np.float32):
    r = np.random.default_rng(seed)
    t = np.arange(n) / max(n, 1)
    x = np.zeros(n)
    for _ in range(5):
        x += np.sin(2 * np.pi * r.uniform(1, 300) * t + r.uniform(0, 6.28))
    x += 1e-3 * r.standard_normal(n)
    x[(t > 0.2) & (t < 0.27)] = 0.0
    return x.astype(dtype)


# ------------------------------------------------------ small parity grid --

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("block", [8, 16, 32, 64, 128, 256, 512, 1024])
def test_parity_block_sizes(dtype, block):
    x = smooth(200_003, 1, dtype)  # many tiles, ragged last block
    for eb in [1e-2, 1e-4]:
        check_parity(x, eb, "rel", block, "blocks")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("eb", [1e-1, 1e-3, 1e-5, 1e-7, 0.0])
def test_parity_error_bounds(dtype, eb):
    x = smooth(333_331, 2, dtype)
    check_parity(x, eb, "rel", 128, "ebs")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_parity_abs_wide_exponents(dtype):
    r = np.random.default_rng(3)
    x = (r.standard_normal(100_000) * 10.0 ** r.integers(-20, 20, 100_000)).astype(dtype)
    x[::7] = 0.0
    for eb in [1e-25, 1e-3, 1.0]:
        check_parity(x, eb, "abs", 128, "abs")


def test_parity_special_values():
    tiny = np.float32(1.4e-45)
    big = np.finfo(np.float32).max
    vals = [0.0, -0.0, tiny, -tiny, 1e-39, -1e-39, 1e-38, big, -big, 1.0, -1.0]
    r = np.random.default_rng(4)
    x = np.array(r.choice(vals, 50_000), dtype=np.float32)
    x[1000:1300] = np.nan
    x[5000] = np.inf
    x[9000] = -np.inf
    for eb in [0.0, 1e-40, 1e-3]:
        for b in [8, 128]:
            check_parity(x, eb, "abs", b, "special")
    check_parity(x, 1e-3, "rel", 128, "special-rel")


def test_parity_all_nan_and_constant():
    x = np.full(10_000, np.nan, dtype=np.float32)
    check_parity(x, 1e-3, "rel", 128, "all-nan")
    x = np.full((33, 1000), 2.5, dtype=np.float64)
    ref = check_parity(x, 1e-3, "rel", 64, "constant")
    assert sf.parse(ref)["n_nc"] == 0


@pytest.mark.parametrize("n", [0, 1, 7, 8, 9, 127, 128, 129, 2047, 2048, 2049, 4095])
def test_parity_ragged_sizes(n):
    for dtype in (np.float32, np.float64):
        x = smooth(n, 5 + n, dtype)
        check_parity(x, 1e-3, "rel", 128, "ragged")
        check_parity(x, 1e-3, "rel", 8, "ragged8")


def test_parity_multidim_metadata():
    from paper_2201_13020_amd import synth
    x = synth.make("turbulence", (20, 50, 50))
    for eb in [1e-2, 1e-3, 1e-4]:
        ref = check_parity(x, eb, "rel", 128, "turbulence-small")
        assert sf.parse(ref)["dims"] == (20, 50, 50)


def striped(n, seed, dtype):
    """Stripes of random length (500 to 40000 values) that alternate between
    smooth values (tiles that compress several times) and full-entropy noise
    (tiles whose mid bytes nearly fill a tile's worst case)."""
    r = np.random.default_rng(seed)
    x = smooth(n, seed).astype(np.float64)
    i, noisy = 0, bool(r.integers(0, 2))
    while i < n:
        ln = int(r.integers(500, 40_000))
        if noisy:
            x[i:i + ln] = r.uniform(-1.0, 1.0, min(ln, n - i))
        i += ln
        noisy = not noisy
    return x.astype(dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("eb", [1e-3, 1e-6, 1e-12])
def test_parity_ring_pressure(dtype, eb):
    """The encoder keeps a finished tile's mid bytes in its LDS ring while it
    encodes the next tile; a tile whose rows would reach them writes the
    pending tile out first, at whatever row that happens. Striped fields put
    that point everywhere, over many tiles; the stream must equal the
    oracle's byte for byte."""
    n = 1_500_037 if dtype == np.float32 else 800_011
    x = striped(n, 17, dtype)
    ref = check_parity(x, eb, "rel", 128, "striped")
    info = sf.parse(ref)
    assert 0 < info["n_nc"] < info["nblk"]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("block", [8, 128])
def test_parity_ladder_and_raw_escalation(dtype, block):
    """The error-control ladder: with a subnormal absolute bound the first
    rung (K0 kept bits) can fail. The oracle's stream for this field holds
    blocks kept at K0, blocks kept at K0 + 1 and finite blocks stored raw
    with K0 < W (outcomes from the definitions, tests/ladder.py); the GPU
    stream must equal it byte for byte."""
    import ladder
    x, eb = ladder.subnormal_field(dtype, 400, block, 7)
    ref = check_parity(x, eb, "abs", block, "ladder")
    got = ladder.outcomes_of_stream(x, sf.parse(ref))
    W = ladder.spec(dtype)[0]
    assert sum(1 for o, K0 in got if o == "K0+1") >= 40
    assert sum(1 for o, K0 in got if o == "raw" and K0 < W) >= 40
    assert sum(1 for o, K0 in got if o == "K0") >= 40


def test_golden_index_propagation_stream():
    from test_oracle_pins import golden_index_propagation_stream
    stream, want = golden_index_propagation_stream()
    y, st = gpu_decompress(stream)
    assert st == 0
    assert np.array_equal(y.view(np.uint32), want)


def test_decoder_flags_corrupt_streams():
    x = smooth(50_000, 7)
    ref = szref.compress(x, 1e-3, "rel", 128)
    info = sf.parse(ref)
    from paper_2201_13020_amd import szx
    exp = szx.inspect(ref[:96].tobytes())
    # bad K byte
    c = ref.copy()
    c[info["offsets"]["K"]] = 5
    y, st = gpu_decompress(c, exp)
    assert st == 3
    # truncated stream (declared size larger than the buffer)
    y, st = gpu_decompress(ref[: len(ref) - 10], exp)
    assert st == 3
    # code larger than the kept bytes: find a block with nb == 2 if any, else flip magic
    c = ref.copy()
    c[0] ^= 0xFF
    y, st = gpu_decompress(c, exp)
    assert st == 3
    # a wrong mid_total
    c = ref.copy()
    c[88] ^= 1
    y, st = gpu_decompress(c, exp)
    assert st == 3
    # the clean stream still decodes
    y, st = gpu_decompress(ref, exp)
    assert st == 0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_decoder_flags_codes_above_kept_bytes(dtype):
    """A code of 3 in a block that keeps only two bytes (nb = 2) is malformed:
    the decoder reports it (and reads nothing outside its buffers)."""
    x = np.cumsum(np.random.default_rng(3).standard_normal(20_000)).astype(dtype)
    ref = szref.compress(x, 1e-2, "rel", 128)
    info = sf.parse(ref)
    from paper_2201_13020_amd import szx
    exp = szx.inspect(ref[:96].tobytes())
    blocks = np.nonzero(info["state"])[0]  # block of each rank
    two = [r for r in range(info["n_nc"]) if info["K"][r] != 0xFF and (int(info["K"][r]) + 7) // 8 == 2
           and sf.block_len(info, int(blocks[r])) == info["b"]]
    assert len(two) > 10
    for r, span in ((two[0], slice(None)), (two[len(two) // 2], slice(5, 6)), (two[-1], slice(31, 32))):
        c = ref.copy()
        row = info["offsets"]["codes"] + r * (info["b"] // 4)
        c[row:row + info["b"] // 4][span] = 0xFF
        y, st = gpu_decompress(c, exp)
        assert st == 3, (r, span)
    y, st = gpu_decompress(ref, exp)
    assert st == 0 and same_bits(y, szref.decompress(ref))


def test_side_stream_while_current_stream_allocates():
    """Calls on a side stream while torch's current stream allocates and
    writes memory: the buffers the binding makes belong to the side stream,
    so nothing it still uses is handed out again. Results equal the oracle."""
    from paper_2201_13020_amd import szx
    x_np = smooth(2_000_003, 11)
    x = torch.from_numpy(x_np).cuda()
    ref = szref.compress(x_np, 1e-3, "rel", 128)
    yref = szref.decompress(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    exp = dict(dtype=torch.float32, dims=tuple(x.shape), block=128)
    for rep in range(3):
        out, size = szx.compress(x, 1e-3, "rel", 128, stream=s)
        churn = [torch.full((1 << 20,), rep + 1, dtype=torch.uint8, device="cuda") for _ in range(32)]
        del churn
        y, st = szx.decompress(out, out.numel(), exp, stream=s)
        churn = [torch.full((1 << 20,), 0xFF, dtype=torch.uint8, device="cuda") for _ in range(32)]
        del churn
        s.synchronize()
        n = int(size.cpu().view(torch.int64).item())
        assert np.array_equal(out[:n].cpu().numpy(), ref), f"rep {rep}"
        assert int(st.cpu().view(torch.int32).item()) == 0
        assert same_bits(y.cpu().numpy(), yref), f"rep {rep}"


def test_determinism_repeated_calls():
    x = smooth(1_000_003, 8)
    a = gpu_roundtrip(x, 1e-3, "rel", 128)[0]
    for _ in range(3):
        b = gpu_roundtrip(x, 1e-3, "rel", 128)[0]
        assert np.array_equal(a, b)


# ------------------------------------------------- full-size workloads --

def test_parity_sines_full():
    from paper_2201_13020_amd import synth
    x = synth.make("sines")
    check_parity(x, 1e-3, "rel", 128, "sines")


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
def test_parity_turbulence_full(eb):
    from paper_2201_13020_amd import synth
    x = synth.make("turbulence")
    check_parity(x, eb, "rel", 128, "turbulence")


@pytest.mark.parametrize("eb", [1e-3, 1e-5])
def test_parity_sphere_full(eb):
    from paper_2201_13020_amd import synth
    x = synth.make("sphere")
    check_parity(x, eb, "rel", 128, "sphere")


def test_graph_replays_match_eager():
    """The C ABI is allocation-free and sync-free, so a compress + decompress
    pair captures into a HIP graph; every replay must match the eager call,
    with other eager work and synchronisations between the replays."""
    from paper_2201_13020_amd import szx
    x_np = smooth(300_001, 9)
    other_np = smooth(120_000, 10)
    x = torch.from_numpy(x_np).cuda()
    other = torch.from_numpy(other_np).cuda()
    cap = szx.compress_bound(torch.float32, x.shape, 1e-3, "rel", 128)
    wsz = szx.workspace_size(torch.float32, x.shape, 1e-3, "rel", 128)
    out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    size = torch.zeros(1, dtype=torch.uint64, device="cuda")
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    st = torch.zeros(1, dtype=torch.uint32, device="cuda")
    exp = dict(dtype=torch.float32, dims=tuple(x.shape), block=128)

    def pair():
        szx.compress(x, 1e-3, "rel", 128, out=out, out_size=size, ws=ws)
        szx.decompress(out, cap, exp, out=y, status=st, ws=ws)

    pair()
    torch.cuda.synchronize()
    n = int(size.cpu().view(torch.int64).item())
    ref_stream = out[:n].cpu().numpy().copy()
    ref_y = y.cpu().numpy().copy()
    assert np.array_equal(ref_stream, szref.compress(x_np, 1e-3, "rel", 128))

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pair()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pair()
    for rep in range(4):
        out.zero_()
        y.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert int(size.cpu().view(torch.int64).item()) == n
        assert np.array_equal(out[:n].cpu().numpy(), ref_stream), f"replay {rep}"
        assert same_bits(y.cpu().numpy(), ref_y), f"replay {rep}"
        assert int(st.cpu().view(torch.int32).item()) == 0
        # unrelated eager work on the same workspace between replays
        o2, s2 = szx.compress(other, 1e-2, "rel", 64)
        torch.cuda.synchronize()


_STATE = {}


def _state():
    if "x" not in _STATE:
        from paper_2201_13020_amd import synth
        _STATE["x"] = synth.make("state")
    return _STATE["x"]


@pytest.mark.parametrize("eb", [1e-3, 1e-5])
def test_parity_state_full(eb):
    """2^28 float64 values (2 GiB): byte-exact stream and bit-exact values."""
    x = _state()
    ref = check_parity(x, eb, "rel", 128, "state")
    info = sf.parse(ref)
    print(f"[state] eb={eb} CR={x.nbytes / ref.size:.3f} constant blocks "
          f"{1 - info['n_nc'] / info['nblk']:.3f}", flush=True)
