"""One field compressed as contiguous block-range shards on one GPU (each
shard with the whole field's bound, from the gathered shard ranges), then
stitched: the stitched stream must equal the oracle's stream of the whole
field byte for byte, and the shard streams must decode, shard by shard, to
the oracle's values bit for bit."""
import numpy as np
import pytest
import torch

from gpu_util import same_bits
from oracle import szref
from paper_2201_13020_amd import synth, szx

pytestmark = pytest.mark.gpu


def shard_bounds(nblk, G):
    """G contiguous block ranges, boundaries at multiples of 8 blocks."""
    cuts = sorted({min(nblk, 8 * round(i * nblk / G / 8)) for i in range(1, G)} - {0, nblk})
    edges = [0] + cuts + [nblk]
    return list(zip(edges[:-1], edges[1:]))


def sharded(x_np, eb, mode, block, G):
    """(stitched stream as numpy, per-shard (stream tensor, size), shard params, bounds)."""
    field = szx.make_params(x_np.dtype, x_np.shape, eb, mode, block)
    n = x_np.size
    nblk = -(-n // block)
    bounds = shard_bounds(nblk, G)
    x = torch.from_numpy(np.ascontiguousarray(x_np).ravel()).cuda()
    parts = [x[k0 * block:min(n, k1 * block)] for k0, k1 in bounds]
    ranges = torch.empty(2 * len(bounds), dtype=torch.float64, device="cuda")
    for i, xs in enumerate(parts):  # step 1 on every shard's GPU
        szx.field_range(xs, block, out=ranges[2 * i:2 * i + 2])
    shards = [szx.compress_shard(field, k0, k1, xs, ranges) for (k0, k1), xs in zip(bounds, parts)]
    out, size = szx.stitch(field, [o for o, _ in shards])
    torch.cuda.synchronize()
    nbytes = int(size.cpu().view(torch.int64).item())
    return out[:nbytes].cpu().numpy(), shards, [szx.shard_params(field, k0, k1) for k0, k1 in bounds], bounds


def decode_shards(shards, sparams):
    ys = []
    for (o, sz), sp in zip(shards, sparams):
        n = int(sz.cpu().view(torch.int64).item())
        y, st = szx.decompress(o, n, szx.params_dict(sp))
        torch.cuda.synchronize()
        assert int(st.cpu().view(torch.int32).item()) == 0
        ys.append(y.cpu().numpy())
    return np.concatenate(ys)


CASES = [
    ("sines 100003 float32 REL 1e-3 b128", lambda: synth.sines_1d(100003), 1e-3, "rel", 128),
    ("turbulence 20x64x64 float32 REL 1e-4 b64", lambda: synth.turbulence_3d((20, 64, 64)), 1e-4, "rel", 64),
    ("walk 70001 float64 ABS 1e-6 b8", lambda: np.cumsum(np.random.default_rng(13020 + 21).standard_normal(70001)),
     1e-6, "abs", 8),
    ("walk 300000 float64 REL 1e-5 b1024", lambda: np.cumsum(np.random.default_rng(13020 + 22).standard_normal(300000)),
     1e-5, "rel", 1024),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("G", [1, 2, 3, 8])
def test_stitched_shards_equal_the_whole_field(case, G):
    name, make, eb, mode, block = case
    x = make()
    print(f"[shard] {name} G={G}", flush=True)
    ref = szref.compress(x, eb, mode, block)
    got, shards, sparams, _ = sharded(x, eb, mode, block, G)
    assert got.size == ref.size and np.array_equal(got, ref), name
    assert same_bits(decode_shards(shards, sparams), szref.decompress(ref).ravel())


def test_stitch_rejects_shards_that_do_not_make_up_the_field():
    x = synth.sines_1d(50000)
    field = szx.make_params("float32", x.shape, 1e-3, "rel", 128)
    got, shards, _, bounds = sharded(x, 1e-3, "rel", 128, 3)
    assert got.size > 0
    # a shard missing
    _, size = szx.stitch(field, [o for o, _ in shards[:2]])
    torch.cuda.synchronize()
    assert int(size.cpu().view(torch.int64).item()) == 0
    # a shard compressed with its own range: another bound than the others
    k0, k1 = bounds[1]
    xs = torch.from_numpy(x[k0 * 128:k1 * 128]).cuda()
    own = szx.field_range(xs)
    other, _ = szx.compress_shard(field, k0, k1, xs, own)
    _, size = szx.stitch(field, [shards[0][0], other, shards[2][0]])
    torch.cuda.synchronize()
    assert int(size.cpu().view(torch.int64).item()) == 0


def test_range_matches_the_finite_extremes():
    rng = np.random.default_rng(13020 + 23)
    for dt in (np.float32, np.float64):
        x = rng.standard_normal(123457).astype(dt)
        x[17] = np.inf
        x[99] = np.nan
        x[1000] = -np.inf
        r = szx.field_range(torch.from_numpy(x).cuda()).cpu().numpy()
        f = x[np.isfinite(x)]
        assert r[0] == f.min() and r[1] == f.max()
    r = szx.field_range(torch.full((1000,), np.nan, dtype=torch.float32, device="cuda")).cpu().numpy()
    assert r[0] == np.inf and r[1] == -np.inf


@pytest.mark.parametrize("G", [2, 4, 8])
def test_state_vector_shards(G, state_field):
    """The 2^28 float64 state vector (2 GiB) in G shards, REL 1e-3."""
    x, ref, yref = state_field
    got, shards, sparams, _ = sharded(x, 1e-3, "rel", 128, G)
    assert got.size == ref.size and np.array_equal(got, ref), f"G={G}"
    assert same_bits(decode_shards(shards, sparams), yref)
    del shards
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def state_field():
    x = synth.make("state")
    print("[shard] state vector generated", flush=True)
    ref = szref.compress(x, 1e-3, "rel", 128)
    yref = szref.decompress(ref).ravel()
    print("[shard] oracle stream and values ready", flush=True)
    return x, ref, yref
